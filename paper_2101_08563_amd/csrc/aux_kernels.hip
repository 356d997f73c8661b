// Auxiliary FastFCA kernels: double precision log-likelihood, P^{-H} and
// ln|det P|^2 per frequency, the decomposed multichannel Wiener filter, and
// initialization / validation helpers.
#include "device.hpp"
#include "internal.hpp"

namespace ffca {

constexpr double kLnPiD = 1.1447298858494002;  // ln(pi)
constexpr int kAuxThreads = 256;
#define FFCA_MAXN_AUX 16

// ------------------------------------------------------------------ block Gauss-Jordan
// Invert the M x M complex matrix held in A[:, 0:M] of the LDS array
// A[M][2M] (columns M..2M-1 must hold the identity on entry) by Gauss-Jordan
// elimination with partial pivoting, in double precision, using every thread
// of the block (uniform control flow). On return A[:, M:2M] holds the
// inverse. Returns false (uniformly) if a pivot is below tol * max|A|;
// *ldet receives ln|det A|^2.
template <int M>
__device__ bool block_gauss_jordan(double2 (*A)[2 * M], double &ldet, double tol) {
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    __shared__ double2 colk[M];
    double amax2 = 0.0;
    for (int i = 0; i < M * M; ++i) amax2 = fmax(amax2, abs2(ld(A[i / M][i % M])));
    bool ok = (amax2 > 0.0) && (amax2 < INFINITY);
    ldet = 0.0;
    for (int k = 0; k < M && ok; ++k) {
        int p = k;
        double best = abs2(ld(A[k][k]));
        for (int i = k + 1; i < M; ++i) {
            const double a = abs2(ld(A[i][k]));
            if (a > best) {
                best = a;
                p = i;
            }
        }
        if (!(best >= tol * tol * amax2)) {
            ok = false;
            break;
        }
        ldet += log(best);
        __syncthreads();
        if (p != k && tid < 2 * M) {
            const double2 t = A[k][tid];
            A[k][tid] = A[p][tid];
            A[p][tid] = t;
        }
        __syncthreads();
        const cd piv = ld(A[k][k]);
        __syncthreads();
        if (tid < 2 * M) A[k][tid] = st(cdiv(ld(A[k][tid]), piv));
        // snapshot column k (the elimination factors) before any row changes
        if (tid < M) colk[tid] = A[tid][k];
        __syncthreads();
        for (int idx = tid; idx < M * 2 * M; idx += nthr) {
            const int i = idx / (2 * M), j = idx % (2 * M);
            if (i != k) A[i][j] = st(ld(A[i][j]) - ld(colk[i]) * ld(A[k][j]));
        }
        __syncthreads();
    }
    return ok;
}

// One workgroup per frequency: ln|det P|^2 by Gauss-Jordan elimination with
// partial pivoting in double precision; a singular P is recorded in the
// frequency's status and its ln|det P|^2 set to NaN.
template <int M>
__global__ void __launch_bounds__(kAuxThreads) ldet_kernel(const WorkItem *items, double *ldet_out) {
    __shared__ double2 A[M][2 * M];
    const WorkItem &it = items[blockIdx.x];
    const int tid = threadIdx.x;
    for (int i = tid; i < M * 2 * M; i += blockDim.x) {
        const int r = i / (2 * M), c = i % (2 * M);
        A[r][c] = c < M ? it.P[r * M + c] : make_double2(c - M == r ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    double ldet;
    const bool ok = block_gauss_jordan<M>(A, ldet, kPivotTol);
    if (tid == 0) {
        if (!ok) *it.status = ST_SINGULAR;
        ldet_out[blockIdx.x] = ok ? ldet : NAN;
    }
}

// ------------------------------------------------------------------ log-likelihood
// LL_f = ln|det P|^2 - (1/T) sum_{m,t} [ln pi + ln sigma^2 + U / sigma^2]
// (eq:negll with the density constant), every term in double precision.
template <int M>
__global__ void __launch_bounds__(kAuxThreads) loglik_kernel(const WorkItem *items,
                                                             const double *ldet, double *ll_f) {
    __shared__ double2 Ps[M * M];
    __shared__ double lam_s[FFCA_MAXN_AUX * M];
    __shared__ double red[kAuxThreads / 64];
    const WorkItem &it = items[blockIdx.x];
    const int tid = threadIdx.x;
    const int T = it.T, N = it.N;
    if (tid < M * M) Ps[tid] = it.P[tid];
    for (int i = tid; i < N * M; i += blockDim.x) lam_s[i] = static_cast<double>(it.lam[i]);
    __syncthreads();
    double acc = 0.0;
    for (int t = tid; t < T; t += blockDim.x) {
        const float *vt = it.v + static_cast<size_t>(t) * N;
        if (it.z) {
            // block model (Sec. VI): U_mj = w_m^H Xhat_j w_m, Xhat_j from its
            // Hermitian parameters
            const float *zt = it.z + static_cast<size_t>(t) * M * M;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                double u = 0.0;
                int p = M;
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    const double2 a = Ps[r * M + m];
                    u += (a.x * a.x + a.y * a.y) * static_cast<double>(zt[r]);
#pragma unroll
                    for (int c = r + 1; c < M; ++c) {
                        const double2 b = Ps[c * M + m];
                        u += 2.0 * ((a.x * b.x + a.y * b.y) * static_cast<double>(zt[p]) -
                                    (a.x * b.y - a.y * b.x) * static_cast<double>(zt[p + 1]));
                        p += 2;
                    }
                }
                double s2 = 0.0;
                for (int n = 0; n < N; ++n) s2 += static_cast<double>(vt[n]) * lam_s[n * M + m];
                acc += kLnPiD + log(s2) + u / s2;
            }
            continue;
        }
        double xr[M], xi[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float2 v = it.x[static_cast<size_t>(t) * M + r];
            xr[r] = v.x;
            xi[r] = v.y;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            double yr = 0.0, yi = 0.0;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                const double2 p = Ps[r * M + m];
                yr += p.x * xr[r] + p.y * xi[r];
                yi += p.x * xi[r] - p.y * xr[r];
            }
            const double u = yr * yr + yi * yi;
            double s2 = 0.0;
            for (int n = 0; n < N; ++n) s2 += static_cast<double>(vt[n]) * lam_s[n * M + m];
            acc += kLnPiD + log(s2) + u / s2;
        }
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) s += red[w];
        ll_f[blockIdx.x] = ldet[blockIdx.x] - s / static_cast<double>(T);
    }
}

// ------------------------------------------------------------------ MWF (eq:Doclo)
// Grid (ceil(Tx / blockDim), F). One thread per TF bin (frame t; its h is
// that of block t / B):
//   z = P^H x ;  for each n: y_n = B (g_n .* z),  g_nm = h_n lam_nm / sigma^2_m,
// with B = P^{-H}. Every workgroup inverts its frequency's P itself (double
// precision Gauss-Jordan in LDS, a few microseconds that overlap across the
// grid) instead of reading it from a separate inversion launch; a singular P
// is recorded in the frequency's status by the workgroup of its first tile.
// M = 2 without LDS or barriers: every thread forms P^{-1} = adj(P) / det P
// in double precision from the frequency's P (the same pivot tests as the
// elimination: the larger entry of column 0, then det P over it, against tol
// times the largest entry), and reads lambda directly.
__global__ void __launch_bounds__(kAuxThreads) mwf2_kernel(const WorkItem *items, int F, float2 *y) {
    const int f = blockIdx.y;
    const WorkItem &it = items[f];
    const int T = it.Tx, N = it.N;
    const cd p00 = ld(it.P[0]), p01 = ld(it.P[1]), p10 = ld(it.P[2]), p11 = ld(it.P[3]);
    const double amax2 = fmax(fmax(abs2(p00), abs2(p01)), fmax(abs2(p10), abs2(p11)));
    const double c0 = fmax(abs2(p00), abs2(p10));
    const cd det = p00 * p11 - p01 * p10;
    const double tol2 = kPivotTol * kPivotTol;
    if (!(amax2 > 0.0) || !(amax2 < INFINITY) || !(c0 >= tol2 * amax2) || !(abs2(det) >= tol2 * amax2 * c0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *it.status = ST_SINGULAR;
        return;
    }
    const cd id = rcp_d(abs2(det)) * conjd(det);
    // B[r][c] = conj(P^{-1}[c][r]); P^{-1} = [[p11, -p01], [-p10, p00]] / det
    const cd b00 = conjd(p11 * id), b01 = conjd(cmk(0.0, 0.0) - p10 * id);
    const cd b10 = conjd(cmk(0.0, 0.0) - p01 * id), b11 = conjd(p00 * id);
    const float2 Pf[4] = {make_float2(static_cast<float>(p00.re), static_cast<float>(p00.im)),
                          make_float2(static_cast<float>(p01.re), static_cast<float>(p01.im)),
                          make_float2(static_cast<float>(p10.re), static_cast<float>(p10.im)),
                          make_float2(static_cast<float>(p11.re), static_cast<float>(p11.im))};
    const float2 Bf[4] = {make_float2(static_cast<float>(b00.re), static_cast<float>(b00.im)),
                          make_float2(static_cast<float>(b01.re), static_cast<float>(b01.im)),
                          make_float2(static_cast<float>(b10.re), static_cast<float>(b10.im)),
                          make_float2(static_cast<float>(b11.re), static_cast<float>(b11.im))};
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    constexpr int M = 2;
    float2 x[M];
#pragma unroll
    for (int r = 0; r < M; ++r) x[r] = it.x[static_cast<size_t>(t) * M + r];
    float2 z[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float zr = 0.f, zi = 0.f;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float2 p = Pf[r * M + m];
            zr = fmaf(p.x, x[r].x, fmaf(p.y, x[r].y, zr));
            zi = fmaf(p.x, x[r].y, fmaf(-p.y, x[r].x, zi));
        }
        z[m] = make_float2(zr, zi);
    }
    const float *vt = it.v + static_cast<size_t>(t / it.B) * N;
    const float *lam = it.lam;
    float rs[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float s = 0.f;
        for (int n = 0; n < N; ++n) s = fmaf(vt[n], lam[n * M + m], s);
        rs[m] = rcp(s);
    }
    for (int n = 0; n < N; ++n) {
        const float vn = vt[n];
        float2 gz[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float g = vn * lam[n * M + m] * rs[m];
            gz[m] = make_float2(g * z[m].x, g * z[m].y);
        }
        float2 *yo = y + ((static_cast<size_t>(n) * F + f) * T + t) * M;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            float ar = 0.f, ai = 0.f;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const float2 b = Bf[r * M + c];
                ar = fmaf(b.x, gz[c].x, fmaf(-b.y, gz[c].y, ar));
                ai = fmaf(b.x, gz[c].y, fmaf(b.y, gz[c].x, ai));
            }
            yo[r] = make_float2(ar, ai);
        }
    }
}

template <int M>
__global__ void __launch_bounds__(kAuxThreads) mwf_kernel(const WorkItem *items, int F, float2 *y) {
    __shared__ double2 A[M][2 * M];
    __shared__ float2 Ps[M * M];
    __shared__ float2 Bs[M * M];
    __shared__ float lam_s[FFCA_MAXN_AUX * M];
    const int f = blockIdx.y;
    const WorkItem &it = items[f];
    const int tid = threadIdx.x;
    const int T = it.Tx, N = it.N;
    for (int i = tid; i < M * 2 * M; i += blockDim.x) {
        const int r = i / (2 * M), c = i % (2 * M);
        A[r][c] = c < M ? it.P[r * M + c] : make_double2(c - M == r ? 1.0 : 0.0, 0.0);
    }
    if (tid < M * M) {
        const double2 p = it.P[tid];
        Ps[tid] = make_float2(static_cast<float>(p.x), static_cast<float>(p.y));
    }
    for (int i = tid; i < N * M; i += blockDim.x) lam_s[i] = it.lam[i];
    __syncthreads();
    double ldet;
    if (!block_gauss_jordan<M>(A, ldet, kPivotTol)) {
        if (blockIdx.x == 0 && tid == 0) *it.status = ST_SINGULAR;
        return;
    }
    // B[r][c] = conj(Pinv[c][r])
    if (tid < M * M) {
        const double2 v = A[tid % M][M + tid / M];
        Bs[tid] = make_float2(static_cast<float>(v.x), static_cast<float>(-v.y));
    }
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + tid;
    if (t >= T) return;
    float2 x[M];
#pragma unroll
    for (int r = 0; r < M; ++r) x[r] = it.x[static_cast<size_t>(t) * M + r];
    float2 z[M];
    float rs[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float zr = 0.f, zi = 0.f;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float2 p = Ps[r * M + m];
            zr = fmaf(p.x, x[r].x, fmaf(p.y, x[r].y, zr));
            zi = fmaf(p.x, x[r].y, fmaf(-p.y, x[r].x, zi));
        }
        z[m] = make_float2(zr, zi);
    }
    const float *vt = it.v + static_cast<size_t>(t / it.B) * N;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float s = 0.f;
        for (int n = 0; n < N; ++n) s = fmaf(vt[n], lam_s[n * M + m], s);
        rs[m] = rcp(s);
    }
    for (int n = 0; n < N; ++n) {
        const float vn = vt[n];
        float2 gz[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float g = vn * lam_s[n * M + m] * rs[m];
            gz[m] = make_float2(g * z[m].x, g * z[m].y);
        }
        float2 *yo = y + ((static_cast<size_t>(n) * F + f) * T + t) * M;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            float ar = 0.f, ai = 0.f;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const float2 b = Bs[r * M + c];
                ar = fmaf(b.x, gz[c].x, fmaf(-b.y, gz[c].y, ar));
                ai = fmaf(b.x, gz[c].y, fmaf(b.y, gz[c].x, ai));
            }
            yo[r] = make_float2(ar, ai);
        }
    }
}

// ------------------------------------------------------------------ helpers
__global__ void check_finite_x_kernel(const float2 *x, size_t n, int *flag) {
    bool bad = false;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const float2 v = x[i];
        bad = bad || !(fabsf(v.x) < INFINITY) || !(fabsf(v.y) < INFINITY);
    }
    if (bad) atomicOr(flag, 1);
}

__global__ void check_positive_kernel(const float *a, size_t n, int *flag) {
    bool bad = false;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const float v = a[i];
        bad = bad || !(v > 0.0f) || !(v < INFINITY);
    }
    if (bad) atomicOr(flag, 1);
}

__global__ void identity_P_kernel(double2 *P, int F, int M) {
    const size_t n = static_cast<size_t>(F) * M * M;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int e = static_cast<int>(i % (static_cast<size_t>(M) * M));
        P[i] = make_double2(e / M == e % M ? 1.0 : 0.0, 0.0);
    }
}

__global__ void fill_int_kernel(int *p, int n, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// fastfca_set_params in one launch: copy P, lambda and v (each optional) and
// clear the frequencies' status. Grid-stride over 16-byte words when both
// pointers of an array are 16-byte aligned, elements otherwise.
template <typename T>
__device__ __forceinline__ void copy_array(T *dst, const T *src, size_t n, size_t i0, size_t stride) {
    if (!dst || !src) return;
    const size_t bytes = n * sizeof(T);
    if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) == 0) {
        const size_t n16 = bytes / 16;
        float4 *d = reinterpret_cast<float4 *>(dst);
        const float4 *s = reinterpret_cast<const float4 *>(src);
        for (size_t i = i0; i < n16; i += stride) d[i] = s[i];
        const size_t done = n16 * 16 / sizeof(T);
        for (size_t i = done + i0; i < n; i += stride) dst[i] = src[i];
    } else {
        for (size_t i = i0; i < n; i += stride) dst[i] = src[i];
    }
}

__global__ void set_params_kernel(double2 *P, const double2 *Ps, size_t nP, float *lam, const float *ls, size_t nl,
                                  float *v, const float *vs, size_t nv, int *status, int F) {
    const size_t i0 = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    copy_array(P, Ps, nP, i0, stride);
    copy_array(lam, ls, nl, i0, stride);
    copy_array(v, vs, nv, i0, stride);
    for (size_t i = i0; i < static_cast<size_t>(F); i += stride) status[i] = ST_OK;
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the k-th output of the stream
// seeded with s is mix(s + (k + 1) * 0x9E3779B97F4A7C15).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double unif24(uint64_t seed, uint64_t k) {
    return static_cast<double>(splitmix64_at(seed, k) >> 40) * (1.0 / 16777216.0);
}

// One workgroup per frequency. lambda_nm = 0.5 + u;
// v_tn = (|x_t|^2/(MN) + d_f)(0.5 + u'), d_f = 1e-6 mean_t |x_t|^2/(MN).
__global__ void __launch_bounds__(kAuxThreads) seeded_init_kernel(const float2 *x, const float *z,
                                                                  float *lam, float *v, int T, int M,
                                                                  int N, uint64_t seed, int do_lam,
                                                                  int do_v) {
    __shared__ double red[kAuxThreads / 64];
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    const double inv_mn = 1.0 / (static_cast<double>(M) * N);
    if (do_lam) {
        for (int i = tid; i < N * M; i += blockDim.x)
            lam[static_cast<size_t>(f) * N * M + i] = static_cast<float>(
                0.5 + unif24(seed, static_cast<uint64_t>(f) * N * M + i));
    }
    if (!do_v) return;
    const float2 *xf = x + static_cast<size_t>(f) * T * M;
    const float *zf = z ? z + static_cast<size_t>(f) * T * M * M : nullptr;
    // power of bin t: |x_t|^2, or tr(Xhat_t) for a block
    auto power = [&](int t) {
        double p = 0.0;
        for (int r = 0; r < M; ++r) {
            if (zf) {
                p += static_cast<double>(zf[static_cast<size_t>(t) * M * M + r]);
            } else {
                const float2 e = xf[static_cast<size_t>(t) * M + r];
                p += static_cast<double>(e.x) * e.x + static_cast<double>(e.y) * e.y;
            }
        }
        return p;
    };
    double acc = 0.0;
    for (int t = tid; t < T; t += blockDim.x) acc += power(t) * inv_mn;
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) tot += red[w];
    const double d = 1e-6 * tot / static_cast<double>(T);
    for (int t = tid; t < T; t += blockDim.x) {
        const double p = power(t) * inv_mn;
        for (int n = 0; n < N; ++n) {
            const uint64_t k = (1ULL << 40) + (static_cast<uint64_t>(f) * T + t) * N + n;
            v[(static_cast<size_t>(f) * T + t) * N + n] =
                static_cast<float>((p + d) * (0.5 + unif24(seed, k)));
        }
    }
}

// ------------------------------------------------------------------ launchers
#define FFCA_M_SWITCH(M, CALL) \
    switch (M) {               \
        case 2: CALL(2); break; \
        case 3: CALL(3); break; \
        case 4: CALL(4); break; \
        case 5: CALL(5); break; \
        case 6: CALL(6); break; \
        case 7: CALL(7); break; \
        case 8: CALL(8); break; \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_ldet(const WorkItem *items, int n_items, int M, double *ldet, hipStream_t s) {
#define FFCA_CALL(MM) hipLaunchKernelGGL(ldet_kernel<MM>, dim3(n_items), dim3(64), 0, s, items, ldet)
    FFCA_M_SWITCH(M, FFCA_CALL)
#undef FFCA_CALL
    return hipGetLastError();
}

hipError_t launch_loglik_terms(const WorkItem *items, int n_items, int M, const double *ldet,
                               double *ll_f, hipStream_t s) {
#define FFCA_CALL(MM) \
    hipLaunchKernelGGL(loglik_kernel<MM>, dim3(n_items), dim3(kAuxThreads), 0, s, items, ldet, ll_f)
    FFCA_M_SWITCH(M, FFCA_CALL)
#undef FFCA_CALL
    return hipGetLastError();
}

hipError_t launch_mwf_bins(const WorkItem *items, int F, int T, int M, float2 *y, hipStream_t s) {
    dim3 grid((T + kAuxThreads - 1) / kAuxThreads, F);
    if (M == 2) {
        hipLaunchKernelGGL(mwf2_kernel, grid, dim3(kAuxThreads), 0, s, items, F, y);
        return hipGetLastError();
    }
#define FFCA_CALL(MM) hipLaunchKernelGGL(mwf_kernel<MM>, grid, dim3(kAuxThreads), 0, s, items, F, y)
    FFCA_M_SWITCH(M, FFCA_CALL)
#undef FFCA_CALL
    return hipGetLastError();
}

static int grid_for(size_t n, int threads) {
    size_t g = (n + threads - 1) / threads;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

hipError_t launch_check_finite_x(const float2 *x, size_t n, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(check_finite_x_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, n, flag);
    return hipGetLastError();
}

hipError_t launch_check_positive(const float *a, size_t n, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(check_positive_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, a, n, flag);
    return hipGetLastError();
}

hipError_t launch_identity_P(double2 *P, int F, int M, hipStream_t s) {
    const size_t n = static_cast<size_t>(F) * M * M;
    hipLaunchKernelGGL(identity_P_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, P, F, M);
    return hipGetLastError();
}

hipError_t launch_set_params(double2 *P, const double2 *Ps, size_t nP, float *lam, const float *ls, size_t nl,
                             float *v, const float *vs, size_t nv, int *status, int F, hipStream_t s) {
    // enough 16-byte words in flight to stream v at full bandwidth; at most 2048 workgroups
    const size_t words = (nv * sizeof(float) + 15) / 16 + static_cast<size_t>(F);
    const int blocks = static_cast<int>(std::min<size_t>(2048, std::max<size_t>(1, (words + 255) / 256)));
    hipLaunchKernelGGL(set_params_kernel, dim3(blocks), dim3(256), 0, s, P, Ps, nP, lam, ls, nl, v, vs, nv, status, F);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int n, int value, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

hipError_t launch_seeded_init(const float2 *x, const float *z, float *lam, float *v, int F, int T,
                              int M, int N, uint64_t seed, bool do_lam, bool do_v, hipStream_t s) {
    hipLaunchKernelGGL(seeded_init_kernel, dim3(F), dim3(kAuxThreads), 0, s, x, z, lam, v, T, M, N,
                       seed, do_lam ? 1 : 0, do_v ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------------ warm start
// Whitening-only start: lambda = 1 and every source gets an equal share of
// the whitened power, v_tn = (1/(M N)) sum_m |(P0^H x_t)_m|^2, with P0 the
// whitening matrix already stored in P. One thread per frame.
template <int M>
__global__ void ws_whitened_kernel(const float2 *x, const double2 *P, float *lam, float *v, int T, int N) {
    const int f = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ float2 Pw[M * M];
    if (threadIdx.x < M * M) {
        const double2 a = P[static_cast<size_t>(f) * M * M + threadIdx.x];
        Pw[threadIdx.x] = make_float2(static_cast<float>(a.x), static_cast<float>(a.y));
    }
    if (blockIdx.x == 0 && static_cast<int>(threadIdx.x) < N * M) lam[static_cast<size_t>(f) * N * M + threadIdx.x] = 1.0f;
    __syncthreads();
    if (t >= T) return;
    const float2 *xt = x + (static_cast<size_t>(f) * T + t) * M;
    float2 xv[M];
#pragma unroll
    for (int r = 0; r < M; ++r) xv[r] = xt[r];
    float pw = 0.0f;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float yr = 0.0f, yi = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float2 a = Pw[r * M + m];
            yr = fmaf(a.x, xv[r].x, fmaf(a.y, xv[r].y, yr));
            yi = fmaf(a.x, xv[r].y, fmaf(-a.y, xv[r].x, yi));
        }
        pw = fmaf(yr, yr, fmaf(yi, yi, pw));
    }
    const float share = pw / static_cast<float>(M * N);
    float *vt = v + (static_cast<size_t>(f) * T + t) * N;
    for (int n = 0; n < N; ++n) vt[n] = share;
}

hipError_t launch_ws_whitened(const float2 *x, const double2 *P, float *lam, float *v, int F, int T, int M, int N,
                              hipStream_t s) {
    if (N * M > kAuxThreads) return hipErrorInvalidValue;
    dim3 grid((T + kAuxThreads - 1) / kAuxThreads, F);
#define FFCA_CALL(MM) hipLaunchKernelGGL(ws_whitened_kernel<MM>, grid, dim3(kAuxThreads), 0, s, x, P, lam, v, T, N)
    FFCA_M_SWITCH(M, FFCA_CALL)
#undef FFCA_CALL
    return hipGetLastError();
}

// Judge of a warm start, per frequency (each frequency is its own problem):
// the new start stays where its log-likelihood is finite and not below that
// of the start it replaced; elsewhere the saved start is copied back. Counts
// the frequencies that kept the new start. One workgroup per frequency.
__global__ void ws_select_kernel(const double *ll_old, const double *ll_new, double2 *P, float *lam, float *v,
                                 const double2 *P_old, const float *lam_old, const float *v_old, int T, int M,
                                 int N, int *n_taken, int *status, const int *status_old, double *ldet,
                                 const double *ldet_old) {
    const int f = blockIdx.x;
    const double a = ll_old[f], b = ll_new[f];
    const bool take = (b == b) && fabs(b) < INFINITY && b >= a;
    if (take) {
        if (threadIdx.x == 0) atomicAdd(n_taken, 1);
        return;
    }
    const size_t fP = static_cast<size_t>(f) * M * M, fl = static_cast<size_t>(f) * N * M;
    const size_t fv = static_cast<size_t>(f) * T * N;
    for (int i = threadIdx.x; i < M * M; i += blockDim.x) P[fP + i] = P_old[fP + i];
    for (int i = threadIdx.x; i < N * M; i += blockDim.x) lam[fl + i] = lam_old[fl + i];
    for (int i = threadIdx.x; i < T * N; i += blockDim.x) v[fv + i] = v_old[fv + i];
    if (threadIdx.x == 0) {
        if (status) status[f] = status_old[f];
        if (ldet) ldet[f] = ldet_old[f];
    }
}

hipError_t launch_ws_select(const double *ll_old, const double *ll_new, double2 *P, float *lam, float *v,
                            const double2 *P_old, const float *lam_old, const float *v_old, int F, int T, int M,
                            int N, int *n_taken, hipStream_t s, int *status, const int *status_old, double *ldet,
                            const double *ldet_old) {
    hipLaunchKernelGGL(ws_select_kernel, dim3(F), dim3(kAuxThreads), 0, s, ll_old, ll_new, P, lam, v, P_old,
                       lam_old, v_old, T, M, N, n_taken, status, status_old, ldet, ldet_old);
    return hipGetLastError();
}

// The race of two starts (fastfca_warmstart_race): per frequency the
// likelihood after the last of the K iterations of either start, from the
// traces the EM kernel wrote (start B in rows [0, F), start A in rows
// [F, 2F), K entries each); -inf for a frequency whose run stopped with an
// error, so that the other start is kept.
__global__ void race_ll_kernel(const double *trace, int K, const int *st_b, const int *st_a, double *ll_b,
                               double *ll_a, int F) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double b = trace[static_cast<size_t>(f) * K + K - 1];
    const double a = trace[static_cast<size_t>(F + f) * K + K - 1];
    ll_b[f] = (st_b[f] == ST_OK && fabs(b) < INFINITY) ? b : -INFINITY;
    ll_a[f] = (st_a[f] == ST_OK && fabs(a) < INFINITY) ? a : -INFINITY;
}

hipError_t launch_race_ll(const double *trace, int K, const int *st_b, const int *st_a, double *ll_b, double *ll_a,
                          int F, hipStream_t s) {
    hipLaunchKernelGGL(race_ll_kernel, dim3((F + 255) / 256), dim3(256), 0, s, trace, K, st_b, st_a, ll_b, ll_a, F);
    return hipGetLastError();
}

// ------------------------------------------------------------------ block covariances
// Xhat_j = (1/B) sum_b x_{jB+b} x_{jB+b}^H (Sec. VI) as M^2 real parameters:
// the diagonal, then re/im of the upper triangle in row-major order. One
// thread per (block, frequency); double precision accumulation.
__global__ void block_cov_kernel(const float2 *x, float *z, int J, int B, int M) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (j >= J) return;
    const float2 *xb = x + (static_cast<size_t>(f) * J + j) * B * M;
    float *zo = z + (static_cast<size_t>(f) * J + j) * M * M;
    const double inv = 1.0 / static_cast<double>(B);
    for (int r = 0; r < M; ++r) {
        double d = 0.0;
        for (int b = 0; b < B; ++b) {
            const float2 a = xb[static_cast<size_t>(b) * M + r];
            d += static_cast<double>(a.x) * a.x + static_cast<double>(a.y) * a.y;
        }
        zo[r] = static_cast<float>(d * inv);
    }
    int p = M;
    for (int r = 0; r < M; ++r)
        for (int c = r + 1; c < M; ++c) {
            double re = 0.0, im = 0.0;
            for (int b = 0; b < B; ++b) {
                const float2 a = xb[static_cast<size_t>(b) * M + r], e = xb[static_cast<size_t>(b) * M + c];
                // x_r conj(x_c)
                re += static_cast<double>(a.x) * e.x + static_cast<double>(a.y) * e.y;
                im += static_cast<double>(a.y) * e.x - static_cast<double>(a.x) * e.y;
            }
            zo[p] = static_cast<float>(re * inv);
            zo[p + 1] = static_cast<float>(im * inv);
            p += 2;
        }
}

hipError_t launch_block_cov(const float2 *x, float *z, int F, int J, int B, int M, hipStream_t s) {
    dim3 grid((J + 127) / 128, F);
    hipLaunchKernelGGL(block_cov_kernel, grid, dim3(128), 0, s, x, z, J, B, M);
    return hipGetLastError();
}

}  // namespace ffca
