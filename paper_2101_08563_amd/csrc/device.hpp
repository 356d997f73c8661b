// Device helpers for the FastFCA kernels (gfx950, 64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>

namespace ffca {

// ----------------------------------------------------------------- wave sums
// DPP controls (GFX9 encoding): quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror, row_mirror. After the four steps every lane of a 16-lane
// row holds the row sum (bitwise identical in every lane, IEEE addition being
// commutative); the four row sums are then combined in a fixed order.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    long long b = __double_as_longlong(v);
    int lo = dpp_i<CTRL>(static_cast<int>(b & 0xffffffffLL));
    int hi = dpp_i<CTRL>(static_cast<int>(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                (static_cast<unsigned int>(lo)));
}

__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double readlane_d(double v, int l) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffLL), l);
    int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                (static_cast<unsigned int>(lo)));
}

// Sum over each 16-lane row: afterwards every lane of a row holds the row's
// sum, bitwise identical across the row. Every lane must be active.
__device__ __forceinline__ float row_sum(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return v;
}

__device__ __forceinline__ double row_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return v;
}

// Sum over the 64 lanes of a wavefront, complete in lane 63 only: after the
// row sums, row_bcast:15 folds row 0 into row 1 and row 2 into row 3, then
// row_bcast:31 folds row 1 into rows 2 and 3 (rows outside the row mask add
// zero). Order: (r3 + r2) + (r1 + r0).
__device__ __forceinline__ float wave_sum_last(float v) {
    v = row_sum(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));
    return v;
}

__device__ __forceinline__ double wave_sum_last(double v) {
    v = row_sum(v);
    {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x142, 0xA, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x142, 0xA, 0xF, false);
        v += __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
    }
    {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x143, 0xC, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x143, 0xC, 0xF, false);
        v += __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
    }
    return v;
}

// Wavefront sums of four values at once, one per 16-lane row:
//   v_permlane32_swap pairs lane i with lane i + 32 for (a, c) and (b, d),
//   v_permlane16_swap then pairs row 0 with row 1 and row 2 with row 3,
//   and a row sum finishes each value.
// Row 0 (lanes 0-15) ends with the total of a, row 1 with b, row 2 with c,
// row 3 with d, the same bits in every lane of a row. Ten instructions for
// four values where four separate wave sums take about forty. Every lane
// must be active.
__device__ __forceinline__ float wave_sum4_rows(float a, float b, float c, float d) {
    const auto ac = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(c), false, false);
    const auto bd = __builtin_amdgcn_permlane32_swap(__float_as_uint(b), __float_as_uint(d), false, false);
    // lanes 0-31: a (b) summed over lanes i, i + 32; lanes 32-63: c (d)
    const float sac = __uint_as_float(ac[0]) + __uint_as_float(ac[1]);
    const float sbd = __uint_as_float(bd[0]) + __uint_as_float(bd[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(sac), __float_as_uint(sbd), false, false);
    // row 0: a over four lanes, row 1: b, row 2: c, row 3: d
    return row_sum(__uint_as_float(q[0]) + __uint_as_float(q[1]));
}

// The same exchange for double precision values: both 32-bit halves of each
// value move with the same lane permutation.
__device__ __forceinline__ double join_d(unsigned int lo, unsigned int hi) {
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
__device__ __forceinline__ void permlane32_swap_d(double &x, double &y) {
    const unsigned long long bx = static_cast<unsigned long long>(__double_as_longlong(x));
    const unsigned long long by = static_cast<unsigned long long>(__double_as_longlong(y));
    const auto lo = __builtin_amdgcn_permlane32_swap(static_cast<unsigned int>(bx), static_cast<unsigned int>(by),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(static_cast<unsigned int>(bx >> 32),
                                                     static_cast<unsigned int>(by >> 32), false, false);
    x = join_d(lo[0], hi[0]);
    y = join_d(lo[1], hi[1]);
}
__device__ __forceinline__ void permlane16_swap_d(double &x, double &y) {
    const unsigned long long bx = static_cast<unsigned long long>(__double_as_longlong(x));
    const unsigned long long by = static_cast<unsigned long long>(__double_as_longlong(y));
    const auto lo = __builtin_amdgcn_permlane16_swap(static_cast<unsigned int>(bx), static_cast<unsigned int>(by),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(static_cast<unsigned int>(bx >> 32),
                                                     static_cast<unsigned int>(by >> 32), false, false);
    x = join_d(lo[0], hi[0]);
    y = join_d(lo[1], hi[1]);
}
// wave_sum4_rows with every cross-lane add in double precision.
__device__ __forceinline__ double wave_sum4_rows(double a, double b, double c, double d) {
    permlane32_swap_d(a, c);
    permlane32_swap_d(b, d);
    double sac = a + c;
    double sbd = b + d;
    permlane16_swap_d(sac, sbd);
    return row_sum(sac + sbd);
}

// Wavefront sums of V values: value v ends in row v % 4 of out[v / 4]
// (wave_sum4_rows on groups of four, zero-padded). With a double output the
// single precision lane partials are promoted first and the whole
// cross-lane tree runs in double precision.
template <int V, class R>
__device__ __forceinline__ void wave_sums_rows(const float (&x)[V], R (&out)[(V + 3) / 4]) {
#pragma unroll
    for (int g = 0; g < (V + 3) / 4; ++g)
        out[g] = wave_sum4_rows(static_cast<R>(x[4 * g]),
                                static_cast<R>(4 * g + 1 < V ? x[4 * g + 1 < V ? 4 * g + 1 : 0] : 0.0f),
                                static_cast<R>(4 * g + 2 < V ? x[4 * g + 2 < V ? 4 * g + 2 : 0] : 0.0f),
                                static_cast<R>(4 * g + 3 < V ? x[4 * g + 3 < V ? 4 * g + 3 : 0] : 0.0f));
}

// Sum over the 64 lanes of a wavefront; the result is wave-uniform.
// Every lane must be active.
__device__ __forceinline__ float wave_sum(float v) {
    v = row_sum(v);
    return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}

__device__ __forceinline__ double wave_sum(double v) {
    v = row_sum(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Single precision reciprocal (v_rcp_f32, about 1 ulp).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Natural log in single precision from the hardware log2 (v_log_f32) for
// normal positive inputs; used only for the per-iteration likelihood trace.
constexpr float kLn2f = 0.69314718055994531f;
__device__ __forceinline__ float log2_fast(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float ln_fast(float x) { return log2_fast(x) * kLn2f; }

// Double precision 1/x and 1/sqrt(x) from the hardware estimates refined by
// Newton steps (each step squares the relative error; two steps reach full
// double precision from the estimate). For finite, normal, positive x.
__device__ __forceinline__ double rcp_d(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt_d(double x) {
    double y = __builtin_amdgcn_rsq(x);
    // y <- y (3 - x y^2) / 2
    y = y * fma(-0.5 * x, y * y, 1.5);
    y = y * fma(-0.5 * x, y * y, 1.5);
    return y;
}

// ----------------------------------------------------------------- complex fp64
struct cd {
    double re, im;
};
__device__ __forceinline__ cd cmk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
    return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cd operator*(double s, cd a) { return cd{s * a.re, s * a.im}; }
__device__ __forceinline__ cd conjd(cd a) { return cd{a.re, -a.im}; }
__device__ __forceinline__ double abs2(cd a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    // Smith's algorithm: avoids overflow of |b|^2 for large b.
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return cd{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        double r = b.re / b.im, d = b.re * r + b.im;
        return cd{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}
__device__ __forceinline__ cd ld(const double2 &a) { return cd{a.x, a.y}; }
__device__ __forceinline__ double2 st(cd a) { return make_double2(a.re, a.im); }

}  // namespace ffca
