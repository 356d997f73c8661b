// FastFCA IP+EM iteration (Algorithm 1, Sec. IV-E) for wide arrays and long
// frames: M <= 8 microphones, N <= 12 sources, T <= 4096 frames.
//
// One workgroup owns one frequency for every iteration of a call. Per bin,
// h_t and U_t stay in registers (BPT bins per thread); x_t is read again from
// global memory in the two passes that need it (weighted covariances, U),
// because an M = 8, T = 4000 frequency (256 KB of x) does not fit on a CU next
// to its h and U.
//
//   A  sigma^2 = L H from the current L and H (eq:sigmadef) and 1/sigma^2;
//      the M weighted covariances Q_m (eq:wsampcov) as a dense
//      contraction over the frequency's bins: each wavefront stages 64 bins
//      (x_t and 1/sigma^2_t) in LDS and lane (r, c, part) accumulates one
//      Hermitian parameter of all M matrices. Every lane runs the same
//      instructions: the imaginary part of x_r conj(x_c) is the real part of
//      x_r conj(i x_c), so those lanes read x_c rotated by a select instead
//      of taking a branch. Each 64-bin chunk is summed in single precision,
//      the chunks and the waves in double precision.
//   IP wave 0, double precision (ip_inv.hpp): the inverses of the Q_m and of
//      P from one Gauss-Jordan run, then for m = 1..M in order w_m from
//      Q_m^{-1} and P^{-1} (eq:ip1, eq:ip2), P^{-1} and det P kept current by
//      rank-one updates; the stage region, idle during the IP, holds its LDS
//      work space.
//   B  U_mt = |w_m^H x_t|^2 (eq:Udef).
//   C  for n = 1..N in order: with g = h_n l_nm / sigma^2_m (sigma^2 from the
//      current L and H, sources before n already updated) the posterior power
//      over h_n is e_m = l_nm (1 + g (U_m / sigma^2_m - 1)); L[:,n] is the
//      T-mean of e (one reduction of M values and one workgroup barrier), then
//      h_n <- h_n (1/M) sum_m e_m / l_nm,new. sigma^2 is formed again for every
//      source rather than kept: at M = 8, N = 10 its 8 values per bin would
//      not fit in registers next to h and U without spilling. Each wavefront
//      keeps its own LDS copy of L, so an update is seen by the rest of its
//      wavefront without a further barrier. The log-likelihood terms of the
//      new iterate (eq:negll) close the phase, while its U is in registers.
#pragma once

#include "device.hpp"
#include "internal.hpp"
#include "ip_inv.hpp"

namespace ffca {

constexpr int kWideBins = 4096;  // largest T of the wide family (threads * BPT)
constexpr int kWideMaxM = 8;
constexpr int kWideMaxN = 12;
constexpr int kWideWaves = 8;    // at most 512 threads per workgroup
constexpr double kWideLnPi = 1.1447298858494002;

constexpr int kWideStage = 32768;  // floats of per-wavefront scratch (128 KB)
static_assert(2 * ip_inv_scratch_doubles<kWideMaxM>() <= kWideStage, "IP scratch in the stage region");

struct WideSmem {
    // per-wavefront scratch, kWideStage / (number of waves) floats each:
    // phase A: staged x (64 bins x M complex), 1/sigma^2 (64 x M), and the
    //          wavefront's double precision partial sums of the Q_m;
    // phase B: staged x and U (64 x M);
    // phase C: the posterior powers e of its bins ([BPT][M][64]).
    alignas(16) float stage[kWideStage];
    alignas(16) float red[2][kWideMaxM][kWideWaves];
    alignas(16) double red_d[kWideWaves];
    float lamw[kWideWaves][kWideMaxN * kWideMaxM];
    float lam_new[kWideMaxN * kWideMaxM];  // Algorithm 2: the new L, formed once for every wave
    double qtot[kWideMaxM * kWideMaxM * kWideMaxM];
    double2 Pd[kWideMaxM * kWideMaxM];
    float2 P32[kWideMaxM * kWideMaxM];
    int flag;
};

// Floats of per-wavefront scratch a launch needs: phase A's staging and
// double precision partials, or phase C's posterior powers.
template <int M, int BPT>
constexpr int wide_region_floats() {
    constexpr int a = 64 * M * 3 + 2 * (64 / (M * M)) * M * M * M;
    constexpr int c = BPT * M * 64;
    return a > c ? a : c;
}

// x_t of bin t (zero for a bin past the end). The frames sit in global
// memory: loads through the global address space compile to global_load,
// where a plain pointer read from the work item gives flat_load, whose
// completion the next LDS wait would also wait for. A bin past the end reads
// bin 0 (T >= 1) and discards it. Callers add an opaque zero to t inside
// their loop over the bins: hoisted out of the iteration loop, the addresses
// of all the bins would be kept (and spilled) across it.
typedef float wf2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) wf2 *gx_ptr;
template <int M>
__device__ __forceinline__ void load_bins(gx_ptr x, int t, int T, float2 (&out)[M]) {
    const bool valid = t < T;
    const unsigned idx = valid ? static_cast<unsigned>(t) * M : 0u;
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const wf2 v = x[idx + r];
        out[r] = valid ? make_float2(v.x, v.y) : make_float2(0.f, 0.f);
    }
}

// MM: Algorithm 2's update of L and H in phase C instead of Algorithm 1's (a
// separate instance, so that each update's register allocation is its own).
template <int M, int N, int BPT, bool MM>
__device__ __forceinline__ void em_wide_item(const WorkItem &it, int n_iter, double alarm, int trace_off,
                                             WideSmem &sm) {
    constexpr int M2 = M * M;
    constexpr int G = 64 / M2;  // lane groups in the weighted-covariance pass
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int nw = nthr >> 6;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int T = it.T;
    const float invTf = 1.0f / static_cast<float>(T);
    const double invT = 1.0 / static_cast<double>(T);
    const gx_ptr xg = (gx_ptr)it.x;  // read once: later global stores could alias the work item

    float vr[BPT][N];
    float U[BPT][M];
    unsigned vmask = 0;  // bit k: bin tid + k * nthr exists
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int t = tid + k * nthr;
        const bool valid = t < T;
        vmask |= valid ? (1u << k) : 0u;
#pragma unroll
        for (int n = 0; n < N; ++n) vr[k][n] = valid ? it.v[t * N + n] : 1.0f;
#pragma unroll
        for (int m = 0; m < M; ++m) U[k][m] = 0.0f;
    }
    float *lamw = sm.lamw[wid];
    for (int i = lane; i < N * M; i += 64) lamw[i] = it.lam[i];
    if (tid < M2) {
        const double2 p = it.P[tid];
        sm.Pd[tid] = p;
        sm.P32[tid] = make_float2(static_cast<float>(p.x), static_cast<float>(p.y));
    }
    for (int i = tid; i < 2 * kWideMaxM * kWideWaves; i += nthr) (&sm.red[0][0][0])[i] = 0.0f;
    if (tid == 0) sm.flag = ST_OK;
    __syncthreads();

    // this lane's Hermitian parameter in the weighted-covariance pass:
    // entry (er, ec); the diagonal |x_r|^2, then re and im of x_r conj(x_c)
    const int grp = lane / M2;
    const int e = lane % M2;
    const bool active = grp < G;
    int er = 0, ec = 0;
    bool rot = false;  // imaginary part: read x_c as i x_c
    if (e < M) {
        er = ec = e;
    } else {
        upper_pair<M>((e - M) >> 1, er, ec);
        rot = ((e - M) & 1) != 0;
    }
    const int region = kWideStage / nw;
    float *stg = sm.stage + wid * region;
    float2 *xs = reinterpret_cast<float2 *>(stg);               // [64][M]
    float *ws = stg + 64 * M * 2;                               // [64][M]
    double *qd = reinterpret_cast<double *>(stg + 64 * M * 3);  // [G][M][M2] partials of this wave

    double ldet_prev = 0.0;
    double ll_last = 0.0;  // LL of the previous iterate (wave 0)
    double lterm = 0.0;    // this lane's ln sigma^2 + U / sigma^2 of the latest iterate
    int buf = 0;
    int status = ST_OK;
    for (int iter = 0; iter <= n_iter; ++iter) {
        const bool last = (iter == n_iter);
        // ---------------- phase A: sigma^2, Q_m. The x of a group of bins is
        // requested before the group's weights 1/sigma^2 are formed.
        if (!last && active) {
#pragma unroll
            for (int m = 0; m < M; ++m) qd[(grp * M + m) * M2 + e] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const bool valid = (vmask >> k) & 1u;
            int loff = 0;
            asm volatile("" : "+v"(loff));
            float2 xk[M];
            if (!last) load_bins<M>(xg, tid + k * nthr + loff, T, xk);
            if (!last) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    float s = 0.0f;
#pragma unroll
                    for (int n = 0; n < N; ++n) s = fmaf(vr[k][n], lamw[loff + n * M + m], s);
                    ws[lane * M + m] = valid ? rcp(s) : 0.0f;
                }
#pragma unroll
                for (int r = 0; r < M; ++r) xs[lane * M + r] = xk[r];
                if (active) {
                    float acc[M];
#pragma unroll
                    for (int m = 0; m < M; ++m) acc[m] = 0.0f;
#pragma unroll 4
                    for (int b = grp; b < 64; b += G) {
                        const float2 xa = xs[b * M + er];
                        const float2 xc = xs[b * M + ec];
                        const float bx = rot ? -xc.y : xc.x;
                        const float by = rot ? xc.x : xc.y;
                        const float z = fmaf(xa.x, bx, xa.y * by);
                        const float *wb = ws + b * M;
#pragma unroll
                        for (int m = 0; m < M; ++m) acc[m] = fmaf(z, wb[m], acc[m]);
                    }
                    // the chunk's single precision sums, added in double precision
#pragma unroll
                    for (int m = 0; m < M; ++m) qd[(grp * M + m) * M2 + e] += static_cast<double>(acc[m]);
                }
            }
            // keep the next bin's loads from being hoisted (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
        asm volatile("" ::: "memory");  // phase boundary: no code motion across it (registers)
        {
            const double l = wave_sum(lterm);
            if (lane == 0) sm.red_d[wid] = l;
        }
        __syncthreads();
        if (!last) {
            // Q_m: the double precision partials of every wave and lane group, in order
            for (int j = tid; j < M * M2; j += nthr) {
                double s = 0.0;
                for (int w = 0; w < nw; ++w) {
                    const double *p = reinterpret_cast<const double *>(sm.stage + w * region + 64 * M * 3);
#pragma unroll
                    for (int g = 0; g < G; ++g) s += p[g * M * M2 + j];
                }
                sm.qtot[j] = s * invT;
            }
            __syncthreads();
        }
        asm volatile("" ::: "memory");  // phase boundary: no code motion across it (registers)
        if (wid == 0) {
            if (iter > 0) {
                double s = 0.0;
                for (int w = 0; w < nw; ++w) s += sm.red_d[w];
                const double ll = ldet_prev - static_cast<double>(M) * kWideLnPi - s * invT;
                if (lane == 0) it.ll_trace[trace_off + iter - 1] = ll;
                if (!(ll == ll) || ll == INFINITY || ll == -INFINITY)
                    status = ST_NONFINITE;
                else if (iter > 1 && ll < ll_last - alarm)  // Algorithm 1 never lowers it
                    status = ST_DECREASE;
                ll_last = ll;
            }
            if (!last && status == ST_OK) {
                double ldet = 0.0;
                // the stage region is idle while wave 0 runs the IP
                status = ip_inv<M>(sm.qtot, sm.Pd, sm.P32, reinterpret_cast<double *>(sm.stage), ldet);
                if (status == ST_OK) ldet_prev = ldet;
            }
            if (lane == 0) sm.flag = status;
        }
        if (last) break;
        __syncthreads();
        status = sm.flag;
        asm volatile("" ::: "memory");  // phase boundary: no code motion across it (registers)
        if (status != ST_OK) break;

        // ---------------- phase B: U = |P^H x|^2, staged per wavefront: the
        // owner lanes put 64 bins' x in LDS, lane (slot, m) forms y_m for
        // every (64/M)-th bin with column m of P held in registers, and the
        // owners read their U back.
        {
            constexpr int S = 64 / M;
            const int mb = lane % M, slot = lane / M;
            float2 pcol[M];
#pragma unroll
            for (int r = 0; r < M; ++r) pcol[r] = sm.P32[r * M + mb];
            float *us = stg + 64 * M * 2;  // [64][M]
            float2 xn[M];
            load_bins<M>(xg, tid, T, xn);
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
#pragma unroll
                for (int r = 0; r < M; ++r) xs[lane * M + r] = xn[r];
                if (k + 1 < BPT) {
                    int z = 0;
                    asm volatile("" : "+v"(z));
                    load_bins<M>(xg, tid + (k + 1) * nthr + z, T, xn);
                }
                if (slot < S) {
#pragma unroll 2
                    for (int b = slot; b < 64; b += S) {
                        float yr = 0.0f, yi = 0.0f;
#pragma unroll
                        for (int r = 0; r < M; ++r) {
                            const float2 xv = xs[b * M + r];
                            yr = fmaf(pcol[r].x, xv.x, fmaf(pcol[r].y, xv.y, yr));
                            yi = fmaf(pcol[r].x, xv.y, fmaf(-pcol[r].y, xv.x, yi));
                        }
                        us[b * M + mb] = fmaf(yr, yr, yi * yi);
                    }
                }
#pragma unroll
                for (int m = 0; m < M; ++m) U[k][m] = us[lane * M + m];
                __builtin_amdgcn_sched_barrier(0);
            }
        }

        asm volatile("" ::: "memory");  // phase boundary: no code motion across it (registers)
        if constexpr (MM) {
            // ---------------- phase C (Algorithm 2): MM update of L from the
            // current L and H, then of H with the new L. Per channel m, the
            // wave's sums over its bins of U v / sigma^4 and v / sigma^2 for
            // every source go to its stage region ([M][2N]); one thread per
            // (n, m) adds the waves in order and writes the new l_nm;
            // every wave copies it into its own L.
            float *rmm = stg;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float lc[N];
#pragma unroll
                for (int nn = 0; nn < N; ++nn) lc[nn] = lamw[nn * M + m];
                float acc[2 * N];
#pragma unroll
                for (int i = 0; i < 2 * N; ++i) acc[i] = 0.0f;
#pragma unroll
                for (int k = 0; k < BPT; ++k) {
                    float s = 0.0f;
#pragma unroll
                    for (int nn = 0; nn < N; ++nn) s = fmaf(vr[k][nn], lc[nn], s);
                    const float is = ((vmask >> k) & 1u) ? rcp(s) : 0.0f;
                    const float ua = U[k][m] * is * is;
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        acc[n] = fmaf(ua, vr[k][n], acc[n]);
                        acc[N + n] = fmaf(is, vr[k][n], acc[N + n]);
                    }
                }
                constexpr int NG = (2 * N + 3) / 4;
                float tot[NG];
                wave_sums_rows<2 * N>(acc, tot);
                if ((lane & 15) == 0) {
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        if (4 * g + (lane >> 4) < 2 * N) rmm[m * 2 * N + 4 * g + (lane >> 4)] = tot[g];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
            float *lnew = sm.lam_new;
            for (int i = tid; i < N * M; i += nthr) {
                const int n = i / M, m = i % M;
                float num = 0.0f, den = 0.0f;
                for (int w = 0; w < nw; ++w) {
                    const float *p = sm.stage + w * region + m * 2 * N;
                    num += p[n];
                    den += p[N + n];
                }
                lnew[i] = lamw[i] * sqrtf(num / den);
            }
            __syncthreads();
            bool good = true;
            for (int i = lane; i < N * M; i += 64) {
                const float l = lnew[i];
                good = good && (l > 0.0f) && (l < INFINITY);
                lamw[i] = l;
            }
            if (!__all(good)) {  // the same values in every wave
                status = ST_NONFINITE;
                break;
            }
            // H rule with the new L, local to each bin
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                float num[N], den[N];
#pragma unroll
                for (int n = 0; n < N; ++n) num[n] = den[n] = 0.0f;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    float lc[N];
#pragma unroll
                    for (int nn = 0; nn < N; ++nn) lc[nn] = lamw[nn * M + m];
                    float s = 0.0f;
#pragma unroll
                    for (int nn = 0; nn < N; ++nn) s = fmaf(vr[k][nn], lc[nn], s);
                    const float is = rcp(s);
                    const float ua = U[k][m] * is * is;
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        num[n] = fmaf(lc[n], ua, num[n]);
                        den[n] = fmaf(lc[n], is, den[n]);
                    }
                }
                const bool valid = (vmask >> k) & 1u;
#pragma unroll
                for (int n = 0; n < N; ++n) vr[k][n] = valid ? vr[k][n] * sqrtf(num[n] / den[n]) : 1.0f;
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
        // ---------------- phase C (Algorithm 1): sources in order
#pragma unroll 1
        for (int n = 0; n < N; ++n) {
            float *es = stg;  // [BPT][M][64], lane-contiguous
            float vn[BPT];
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                float a = 0.0f;
#pragma unroll
                for (int nn = 0; nn < N; ++nn) a = (nn == n) ? vr[k][nn] : a;
                vn[k] = a;
            }
            float part[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float lc[N];
#pragma unroll
                for (int nn = 0; nn < N; ++nn) lc[nn] = lamw[nn * M + m];
                const float lo = lamw[n * M + m];
                float pm = 0.0f;
#pragma unroll
                for (int k = 0; k < BPT; ++k) {
                    float s = 0.0f;
#pragma unroll
                    for (int nn = 0; nn < N; ++nn) s = fmaf(vr[k][nn], lc[nn], s);
                    const float a = vn[k] * lo;
                    const float w = rcp(s);
                    const float r = fmaf(U[k][m], w, -1.0f);
                    const float ek = fmaf(lo * (a * w), r, lo);
                    es[(k * M + m) * 64 + lane] = ek;
                    pm += ((vmask >> k) & 1u) ? ek : 0.0f;
                }
                part[m] = pm;
                __builtin_amdgcn_sched_barrier(0);
            }
            {
                constexpr int NG = (M + 3) / 4;
                float tot[NG];
                wave_sums_rows<M>(part, tot);
                if ((lane & 15) == 0) {
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        if (4 * g + (lane >> 4) < M) sm.red[buf][4 * g + (lane >> 4)][wid] = tot[g];
                }
            }
            __syncthreads();
            float lmine = 0.0f;
            if (lane < M) {
                const float *p = sm.red[buf][lane];
#pragma unroll
                for (int w = 0; w < kWideWaves; ++w) lmine += p[w];
                lmine *= invTf;
            }
            buf ^= 1;
            const bool good = __all(lane >= M || ((lmine > 0.0f) && (lmine < INFINITY)));
            if (!good) {
                status = ST_NONFINITE;
                break;
            }
            if (lane < M) lamw[n * M + lane] = lmine;
            float s[BPT];
#pragma unroll
            for (int k = 0; k < BPT; ++k) s[k] = 0.0f;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const float c = rcp(readlane_f(lmine, m) * static_cast<float>(M));
#pragma unroll
                for (int k = 0; k < BPT; ++k) s[k] = fmaf(es[(k * M + m) * 64 + lane], c, s[k]);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const bool valid = (vmask >> k) & 1u;
                const float vnew = valid ? vn[k] * s[k] : 1.0f;
#pragma unroll
                for (int nn = 0; nn < N; ++nn)
                    if (nn == n) vr[k][nn] = vnew;
            }
        }
        }  // Algorithm 1
        if (status != ST_OK) break;
        // log-likelihood terms of the new iterate (eq:negll), reported in the
        // next pass of phase A
        lterm = 0.0;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            float lg = 0.0f, uw = 0.0f;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float s2 = 0.0f;
#pragma unroll
                for (int nn = 0; nn < N; ++nn) s2 = fmaf(vr[k][nn], lamw[nn * M + m], s2);
                lg += log2_fast(s2);
                uw = fmaf(U[k][m], rcp(s2), uw);
            }
            if ((vmask >> k) & 1u)
                lterm += static_cast<double>(lg) * static_cast<double>(kLn2f) + static_cast<double>(uw);
        }
        asm volatile("" ::: "memory");  // phase boundary: no code motion across it (registers)
    }

    if (wid == 0) {
        for (int i = lane; i < N * M; i += 64) it.lam[i] = lamw[i];
        if (lane < M2) it.P[lane] = sm.Pd[lane];
        if (lane == 0) {
            *it.ldet = ldet_prev;
            if (status != ST_OK) *it.status = status;
        }
    }
    // v last: stored after L, P and the status, this block leaves the
    // register allocator with less live across the iteration loop (at
    // M = 8, N = 10, eight bins per thread, 57 spilled VGPRs instead of 138)
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int t = tid + k * nthr;
        if ((vmask >> k) & 1u) {
#pragma unroll
            for (int n = 0; n < N; ++n) it.v[t * N + n] = vr[k][n];
        }
    }
    __syncthreads();
}

}  // namespace ffca
