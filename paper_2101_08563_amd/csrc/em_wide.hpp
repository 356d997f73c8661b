// FastFCA IP+EM iteration (Algorithm 1, Sec. IV-E) for wide arrays and long
// frames: M <= 8 microphones, N <= 12 sources, T <= 4096 frames.
//
// One workgroup owns one frequency for every iteration of a call. Per-bin h_t
// and U_t stay in registers (BPT bins per thread); x_t is read again from
// global memory in the two passes that need it (weighted covariances, U),
// because an M = 8, T = 4000 frequency (256 KB of x) does not fit on a CU
// next to its h and U.
//
//   A  sigma^2 and 1/sigma^2 (eq:sigmadef); the M weighted covariances Q_m
//      (eq:wsampcov) as a dense contraction over the frequency's bins: each
//      wavefront stages 64 bins (x_t, 1/sigma^2_t) in LDS and lane (r, c) of
//      the wavefront accumulates the Hermitian parameter (r, c) of all M
//      matrices (M^2 <= 64 lanes; smaller M use several lane groups on
//      different bins); the log-likelihood terms of the previous iterate.
//   IP wave 0, double precision, one matrix element per lane: for
//      m = 1..M, A = P^H Q_m, Gauss-Jordan elimination with partial pivoting
//      on [A | e_m] (eq:ip1), normalization (eq:ip2); then ln|det P|^2.
//   B  U_mt = |w_m^H x_t|^2 (eq:Udef).
//   C  for n = 1..N in order: G_n, Phi_n, L[:,n] (T-reduction), H[n,:].
//      Each wavefront keeps its own LDS copy of L so an update by one lane is
//      seen by the rest of its wavefront without a workgroup barrier.
#pragma once

#include "device.hpp"
#include "internal.hpp"
#include "ip_wave.hpp"

namespace ffca {

constexpr int kWideBins = 4096;  // largest T of the wide family (threads * BPT)
constexpr int kWideMaxM = 8;
constexpr int kWideMaxN = 12;
constexpr int kWideWaves = 16;
constexpr double kWideLnPi = 1.1447298858494002;

constexpr int kWideStage = 32768;  // floats of per-wavefront scratch (128 KB)

struct WideSmem {
    // per-wavefront scratch, kWideStage / (number of waves) floats each:
    // staged x (64 bins x M complex) and 1/sigma^2 or U (64 x M) in phases A
    // and B, the wavefront's partial sums of the Q_m (64 M floats) after A,
    // and the posterior powers Phi_n of its bins (64 BPT M floats) in C.
    alignas(16) float stage[kWideStage];
    alignas(16) float red[2][kWideMaxM][kWideWaves];
    alignas(16) double red_d[2][kWideWaves];
    float lamw[kWideWaves][kWideMaxN * kWideMaxM];
    double qtot[kWideMaxM * kWideMaxM * kWideMaxM];
    double2 Pd[kWideMaxM * kWideMaxM];
    float2 P32[kWideMaxM * kWideMaxM];
    IpLds<kWideMaxM> ip;
    int flag;
};

template <int M, int N, int BPT>
__device__ __forceinline__ void em_wide_item(const WorkItem &it, int n_iter, double alarm, WideSmem &sm) {
    constexpr int M2 = M * M;
    constexpr int G = 64 / M2;  // lane groups in the weighted-covariance pass
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int T = it.T;
    const float invTf = 1.0f / static_cast<float>(T);
    const double invT = 1.0 / static_cast<double>(T);

    float vr[BPT][N];
    float U[BPT][M];
    bool valid[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int t = tid + k * nthr;
        valid[k] = t < T;
#pragma unroll
        for (int n = 0; n < N; ++n) vr[k][n] = valid[k] ? it.v[t * N + n] : 1.0f;
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
    if (tid < 2 * kWideWaves) (&sm.red_d[0][0])[tid] = 0.0;
    if (tid == 0) sm.flag = ST_OK;
    __syncthreads();

    // this lane's role in the weighted-covariance pass
    const int grp = lane / M2;
    const int e = lane % M2;
    const bool active = grp < G;
    int er = 0, ec = 0, epart = 0;  // entry (r, c); part 0 = |x_r|^2, 1 = re, 2 = im
    if (e < M) {
        er = ec = e;
    } else {
        upper_pair<M>((e - M) >> 1, er, ec);
        epart = 1 + ((e - M) & 1);
    }
    const int region = kWideStage / (nthr >> 6);
    float *stg = sm.stage + wid * region;
    float2 *xs = reinterpret_cast<float2 *>(stg);  // [64][M]
    float *ws = stg + 64 * M * 2;                  // [64][M]

    double ldet_prev = 0.0;
    double ll_last = 0.0;  // LL of the previous iterate (wave 0)
    double llp = 0.0;  // LL terms of the latest iterate (end of phase C)
    int buf = 0;
    int status = ST_OK;
    for (int iter = 0; iter <= n_iter; ++iter) {
        const bool last = (iter == n_iter);
        // ---------------- phase A
        float acc[M];
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] = 0.0f;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int t = tid + k * nthr;
            float2 xk[M];
#pragma unroll
            for (int r = 0; r < M; ++r) xk[r] = valid[k] ? it.x[t * M + r] : make_float2(0.f, 0.f);
            float w[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float s = 0.0f;
#pragma unroll
                for (int n = 0; n < N; ++n) s = fmaf(vr[k][n], lamw[n * M + m], s);
                w[m] = rcp(s);
                if (N > 6) __builtin_amdgcn_sched_barrier(0);
            }
            if (!last) {
#pragma unroll
                for (int r = 0; r < M; ++r) xs[lane * M + r] = xk[r];
#pragma unroll
                for (int m = 0; m < M; ++m) ws[lane * M + m] = valid[k] ? w[m] : 0.0f;
                if (active) {
#pragma unroll 2
                    for (int b = grp; b < 64; b += G) {
                        const float2 xa = xs[b * M + er], xb = xs[b * M + ec];
                        float z;
                        if (epart == 0)
                            z = fmaf(xa.x, xa.x, xa.y * xa.y);
                        else if (epart == 1)
                            z = fmaf(xa.x, xb.x, xa.y * xb.y);
                        else
                            z = fmaf(xa.y, xb.x, -xa.x * xb.y);
                        const float *wb = ws + b * M;
#pragma unroll
                        for (int m = 0; m < M; ++m) acc[m] = fmaf(z, wb[m], acc[m]);
                    }
                }
            }
            // keep the next bin's loads from being hoisted (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
        if (!last && active) {
#pragma unroll
            for (int m = 0; m < M; ++m) stg[(grp * M + m) * M2 + e] = acc[m];
        }
        {
            const double l = wave_sum(llp);
            if (lane == 0) sm.red_d[buf][wid] = l;
        }
        __syncthreads();
        if (!last) {
            const int nw = nthr >> 6;
            for (int j = tid; j < M * M2; j += nthr) {
                float s = 0.0f;
                for (int w = 0; w < nw; ++w)
#pragma unroll
                    for (int g = 0; g < G; ++g) s += sm.stage[w * region + g * M * M2 + j];
                sm.qtot[j] = static_cast<double>(s) * invT;
            }
            __syncthreads();
        }
        if (wid == 0) {
            if (iter > 0) {
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < kWideWaves; ++w) s += sm.red_d[buf][w];
                const double ll = ldet_prev - static_cast<double>(M) * kWideLnPi - s * invT;
                if (lane == 0) it.ll_trace[iter - 1] = ll;
                if (!(ll == ll) || ll == INFINITY || ll == -INFINITY)
                    status = ST_NONFINITE;
                else if (iter > 1 && ll < ll_last - alarm)  // Algorithm 1 never lowers it
                    status = ST_DECREASE;
                ll_last = ll;
            }
            if (!last && status == ST_OK) {
                double ldet = 0.0;
                status = ip_wave<M, kWideMaxM>(sm.qtot, sm.Pd, sm.P32, sm.ip, ldet);
                if (status == ST_OK) ldet_prev = ldet;
            }
            if (lane == 0) sm.flag = status;
        }
        if (last) break;
        __syncthreads();
        status = sm.flag;
        if (status != ST_OK) break;
        buf ^= 1;

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
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const int t = tid + k * nthr;
#pragma unroll
                for (int r = 0; r < M; ++r)
                    xs[lane * M + r] = valid[k] ? it.x[t * M + r] : make_float2(0.f, 0.f);
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

        // ---------------- phase C: sources in order
#pragma unroll 1
        for (int n = 0; n < N; ++n) {
            float *phis = stg;  // [BPT][M][64], lane-contiguous
            float part[M];
            float vn[BPT], rv[BPT];
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                // source n's power without a dynamically indexed register array
                float a = 0.0f;
#pragma unroll
                for (int nn = 0; nn < N; ++nn) a = (nn == n) ? vr[k][nn] : a;
                vn[k] = a;
                rv[k] = valid[k] ? rcp(a) : 0.0f;
            }
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float lc[N];
#pragma unroll
                for (int nn = 0; nn < N; ++nn) lc[nn] = lamw[nn * M + m];
                const float ln_ = lamw[n * M + m];
                float pm = 0.0f;
#pragma unroll
                for (int k = 0; k < BPT; ++k) {
                    float s = 0.0f;
#pragma unroll
                    for (int nn = 0; nn < N; ++nn) s = fmaf(vr[k][nn], lc[nn], s);
                    const float a = vn[k] * ln_;
                    const float g = a * rcp(s);
                    const float ph = fmaf(g * g, U[k][m], (1.0f - g) * a);
                    phis[(k * M + m) * 64 + lane] = ph;
                    pm = fmaf(ph, rv[k], pm);
                }
                part[m] = pm;
                __builtin_amdgcn_sched_barrier(0);
            }
            {
                // wave sums four values at a time, value 4g + r in row r
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
            float s16 = 0.0f;
            if (lane < M) {
                const float *p = sm.red[buf][lane];
#pragma unroll
                for (int w = 0; w < kWideWaves; ++w) s16 += p[w];
            }
            float rl[M];
            bool good = true;
            float lnew_mine = 0.0f;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const float l = readlane_f(s16, m) * invTf;
                good = good && (l > 0.0f) && (l < INFINITY);
                rl[m] = rcp(l);
                if (lane == m) lnew_mine = l;
            }
            buf ^= 1;
            if (!good) {
                status = ST_NONFINITE;
                break;
            }
            if (lane < M) lamw[n * M + lane] = lnew_mine;
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                float s = 0.0f;
#pragma unroll
                for (int m = 0; m < M; ++m) s = fmaf(phis[(k * M + m) * 64 + lane], rl[m], s);
                const float vnew = valid[k] ? s * (1.0f / static_cast<float>(M)) : 1.0f;
#pragma unroll
                for (int nn = 0; nn < N; ++nn)
                    if (nn == n) vr[k][nn] = vnew;
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (status != ST_OK) break;
        // log-likelihood terms of this iterate (eq:negll): final sigma^2, U
        llp = 0.0;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            float lacc = 0.0f;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float s = 0.0f;
#pragma unroll
                for (int n = 0; n < N; ++n) s = fmaf(vr[k][n], lamw[n * M + m], s);
                lacc += ln_fast(s) + U[k][m] * rcp(s);
            }
            if (valid[k]) llp += static_cast<double>(lacc);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (status != ST_OK) break;
    }

#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int t = tid + k * nthr;
        if (valid[k]) {
#pragma unroll
            for (int n = 0; n < N; ++n) it.v[t * N + n] = vr[k][n];
        }
    }
    if (wid == 0) {
        for (int i = lane; i < N * M; i += 64) it.lam[i] = lamw[i];
        if (lane < M2) it.P[lane] = sm.Pd[lane];
        if (lane == 0) {
            *it.ldet = ldet_prev;
            if (status != ST_OK) *it.status = status;
        }
    }
    __syncthreads();
}

}  // namespace ffca
