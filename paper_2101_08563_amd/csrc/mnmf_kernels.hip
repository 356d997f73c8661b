// FastMNMF (Sec. V "FastMNMF: Full-band Extension of FastFCA" and its
// appendix; eq:NMFconst2, eq:FastMNMFcost) on gfx950.
//
// The source powers are an NMF over frequency and time,
//   h_{ijn} = sum_k t_{ikn} v_{jkn},
// so the frequencies share the activations V and one iteration is a
// per-frequency pass followed by a pass over frames:
//
//   mnmf_freq_kernel (one workgroup per frequency i, bins in registers):
//     h from t_i (LDS) and V (global, shared by all workgroups);
//     log-likelihood of the current state (eq:FastMNMFcost);
//     Q_m (eq:wsampcov) and the IP sweep of W_i in double precision (eq:ip1,
//     eq:ip2); U = |w^H x|^2 (eq:Udef);
//     Lambda_i by the multiplicative MM rule (one 2NM-value T-reduction);
//     T_i by the MM rule (2KN values, reduced KC patterns at a time);
//     with the new Lambda_i and t_i: G_ijn = sum_m lambda U / sigma^4 and
//     E_ijn = sum_m lambda / sigma^2 to global memory.
//   mnmf_v_partial_kernel / mnmf_v_update_kernel: for every (j, k, n),
//     v <- v sqrt( sum_i t_ikn G_ijn / sum_i t_ikn E_ijn ), the sum over i
//     split in fixed frequency chunks and combined in a fixed order.
//
// Every MM rule has the form theta <- theta sqrt(sum phi U / sigma^4 /
// sum phi / sigma^2) for the coefficient phi of theta in sigma^2.
#include "em_item.hpp"
#include "mnmf.hpp"

namespace ffca {

template <int M, int N, int NWS>
struct MnmfSmem {
    static constexpr int RC = 2 * kMnmfKC * N > 2 * N * M ? 2 * kMnmfKC * N : 2 * N * M;
    alignas(16) double redq[M * M * M][4 * NWS];  // row partials of the Q_m, double precision
    alignas(16) double red_d[4 * NWS];
    alignas(16) float redc[2][RC][NWS];
    float sums[RC];
    double qtot[M * M * M];
    double2 Pd[kMaxM * kMaxM];
    float2 P32[kMaxM * kMaxM];
    IpSmLds<kMaxM> ip;
    float t[kMnmfKMax * N];
    int flag;
};

template <int M, int N, int BPT>
__global__ void __launch_bounds__(kResidentBins / BPT) mnmf_freq_kernel(MnmfLaunch a) {
    constexpr int NWS = wave_slots(BPT);
    constexpr int NQ = M * M * M;
    constexpr int NR = 4 * NWS;
    constexpr int KC = kMnmfKC;
    __shared__ MnmfSmem<M, N, NWS> sm;
    const int i = blockIdx.x;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const bool row_lead = (lane & 15) == 0;
    const int row_slot = 4 * wid + (lane >> 4);
    const int T = a.T, K = a.K;
    const double invT = 1.0 / static_cast<double>(T);
    const float2 *x = a.x + static_cast<size_t>(i) * T * M;
    float *G = a.G + static_cast<size_t>(i) * T * N;
    float *E = a.E + static_cast<size_t>(i) * T * N;
    auto retire = [&]() {  // a failed frequency adds nothing to the V rule
        if (!a.ll_only)
            for (int q = tid; q < T * N; q += nthr) {
                G[q] = 0.0f;
                E[q] = 0.0f;
            }
    };
    if (a.status[i] != ST_OK) {
        retire();
        return;
    }

    // ---- state
    float2 xr[BPT][M];
    float h[BPT][N];
    float U[BPT][M];
    float mk[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int t = tid + k * nthr;
        const bool valid = t < T;
        mk[k] = valid ? 1.0f : 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) xr[k][r] = valid ? x[t * M + r] : make_float2(0.f, 0.f);
    }
    float lam[N][M];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int m = 0; m < M; ++m) lam[n][m] = a.lam[(static_cast<size_t>(i) * N + n) * M + m];
    for (int q = tid; q < K * N; q += nthr) sm.t[q] = a.tp[static_cast<size_t>(i) * K * N + q];
    if (tid < M * M) {
        const double2 p = a.P[static_cast<size_t>(i) * M * M + tid];
        sm.Pd[tid] = p;
        sm.P32[tid] = make_float2(static_cast<float>(p.x), static_cast<float>(p.y));
    }
    for (int q = tid; q < static_cast<int>(sizeof(sm.redq) / sizeof(double)); q += nthr) (&sm.redq[0][0])[q] = 0.0;
    for (int q = tid; q < static_cast<int>(sizeof(sm.redc) / sizeof(float)); q += nthr) (&sm.redc[0][0][0])[q] = 0.0f;
    for (int q = tid; q < NR; q += nthr) sm.red_d[q] = 0.0;
    if (tid == 0) sm.flag = ST_OK;
    __syncthreads();

    // h_jn = sum_k t_kn v_jkn for this thread's bins (1 for bins t >= T).
    // Bins past T read frame T - 1 and drop it, so no branch splits the
    // loads of the BPT bins and they are all in flight together.
    auto make_h = [&]() {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int t = tid + k * nthr;
            float s[N];
#pragma unroll
            for (int n = 0; n < N; ++n) s[n] = 0.0f;
            const float *vt = a.va + (t < T ? t : T - 1);  // activations stored [K][N][T]
#pragma unroll 8
            for (int kk = 0; kk < K; ++kk)
#pragma unroll
                for (int n = 0; n < N; ++n)
                    s[n] = fmaf(sm.t[kk * N + n], vt[static_cast<size_t>(kk * N + n) * T], s[n]);
#pragma unroll
            for (int n = 0; n < N; ++n) h[k][n] = t < T ? s[n] : 1.0f;
        }
    };
    // U_mt = |w_m^H x_t|^2 with the single precision copy of P
    auto make_U = [&]() {
        float2 Pw[M][M];
#pragma unroll
        for (int q = 0; q < M * M; ++q) Pw[q / M][q % M] = sm.P32[q];
#pragma unroll
        for (int k = 0; k < BPT; ++k)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float yr = 0.0f, yi = 0.0f;
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    yr = fmaf(Pw[r][m].x, xr[k][r].x, yr);
                    yr = fmaf(Pw[r][m].y, xr[k][r].y, yr);
                    yi = fmaf(Pw[r][m].x, xr[k][r].y, yi);
                    yi = fmaf(-Pw[r][m].y, xr[k][r].x, yi);
                }
                U[k][m] = yr * yr + yi * yi;
            }
    };
    auto sigma2 = [&](int k, int m) {
        float s = 0.0f;
#pragma unroll
        for (int n = 0; n < N; ++n) s = fmaf(h[k][n], lam[n][m], s);
        return s;
    };

    make_h();
    make_U();

    // ---- log-likelihood of the current state (written for the iteration before)
    if (a.iter > 0) {
        float lg2 = 0.0f, uw = 0.0f;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            float l = 0.0f;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const float s = sigma2(k, m);
                l += log2_fast(s);
                uw = fmaf(U[k][m], rcp(s), uw);
            }
            lg2 = fmaf(mk[k], l, lg2);
        }
        const double llp = row_sum(static_cast<double>(lg2) * static_cast<double>(kLn2f) + static_cast<double>(uw));
        if (row_lead) sm.red_d[row_slot] = llp;
        __syncthreads();
        if (tid == 0) {
            const double ll = a.ldet[i] - static_cast<double>(M) * kLnPi - sum_slots<NR>(sm.red_d) * invT;
            a.ll_trace[static_cast<size_t>(i) * a.cap + a.iter - 1] = ll;
            if (!(ll == ll) || ll == INFINITY || ll == -INFINITY) a.status[i] = ST_NONFINITE;
        }
        if (a.ll_only) return;
    }

    // ---- Q_m (eq:wsampcov) and the IP sweep (eq:ip1, eq:ip2)
    {
        float q[NQ];
#pragma unroll
        for (int e = 0; e < NQ; ++e) q[e] = 0.0f;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            float z[M * M];
#pragma unroll
            for (int r = 0; r < M; ++r) z[r] = xr[k][r].x * xr[k][r].x + xr[k][r].y * xr[k][r].y;
            int p = M;
#pragma unroll
            for (int r = 0; r < M; ++r)
#pragma unroll
                for (int c = r + 1; c < M; ++c) {
                    z[p] = xr[k][r].x * xr[k][c].x + xr[k][r].y * xr[k][c].y;
                    z[p + 1] = xr[k][r].y * xr[k][c].x - xr[k][r].x * xr[k][c].y;
                    p += 2;
                }
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const float w = rcp(sigma2(k, m));
#pragma unroll
                for (int e = 0; e < M * M; ++e) q[m * M * M + e] = fmaf(w, z[e], q[m * M * M + e]);
            }
        }
        // lane partials are single precision; the sums across lanes and waves
        // are double precision (as in the frame model's kernel)
        double qd[NQ];
#pragma unroll
        for (int e = 0; e < NQ; ++e) qd[e] = row_sum(static_cast<double>(q[e]));
        if (row_lead) {
#pragma unroll
            for (int e = 0; e < NQ; ++e) sm.redq[e][row_slot] = qd[e];
        }
    }
    __syncthreads();
    if (wid == 0) {
        double ldet = 0.0;
        int st;
        if constexpr (M == 2) {
            const cd Pc[4] = {ld(sm.Pd[0]), ld(sm.Pd[1]), ld(sm.Pd[2]), ld(sm.Pd[3])};
            double qs[8];
            const double mine = sum_slots<NR>(sm.redq[lane & 7]);
#pragma unroll
            for (int e = 0; e < 8; ++e) qs[e] = readlane_d(mine, e);
            double det2 = 1.0;
            st = ip_sweep_reg2(sm, Pc, qs, sqrt(static_cast<double>(T)), det2);
            ldet = log(det2);
        } else {
            if (lane < NQ) sm.qtot[lane] = sum_slots<NR>(sm.redq[lane]) * invT;
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
            st = ip_sm<M, kMaxM>(sm.qtot, sm.Pd, sm.P32, sm.ip, ldet);
        }
        if (lane == 0) {
            sm.flag = st;
            if (st == ST_OK) a.ldet[i] = ldet;
        }
    }
    __syncthreads();
    if (sm.flag != ST_OK) {
        if (tid == 0) a.status[i] = sm.flag;
        retire();
        return;
    }
    make_U();

    int buf = 0;
    bool good = true;
    // ---- Lambda_i: phi = h_jn, sums over j
    {
        float nd[2 * N * M];
#pragma unroll
        for (int e = 0; e < 2 * N * M; ++e) nd[e] = 0.0f;
#pragma unroll
        for (int k = 0; k < BPT; ++k)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const float is = mk[k] * rcp(sigma2(k, m));
                const float ua = U[k][m] * is * is;
#pragma unroll
                for (int n = 0; n < N; ++n) {
                    nd[n * M + m] = fmaf(ua, h[k][n], nd[n * M + m]);
                    nd[N * M + n * M + m] = fmaf(is, h[k][n], nd[N * M + n * M + m]);
                }
            }
#pragma unroll
        for (int e = 0; e < 2 * N * M; ++e) nd[e] = wave_sum_last(nd[e]);
        if (lane == 63) {
#pragma unroll
            for (int e = 0; e < 2 * N * M; ++e) sm.redc[buf][e][wid] = nd[e];
        }
        __syncthreads();
        const float mine = lane < 2 * N * M ? sum_slots<NWS>(sm.redc[buf][lane]) : 0.0f;
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const float l = lam[n][m] * sqrtf(readlane_f(mine, n * M + m) / readlane_f(mine, N * M + n * M + m));
                good = good && (l > 0.0f) && (l < INFINITY);
                lam[n][m] = l;
            }
        buf ^= 1;
    }

    // ---- T_i: phi = lambda_imn v_jkn, sums over j and m (sigma^2 from the
    // new Lambda and the old t for every pattern)
    {
        float an[BPT][N], bn[BPT][N];
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
#pragma unroll
            for (int n = 0; n < N; ++n) an[k][n] = bn[k][n] = 0.0f;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const float is = mk[k] * rcp(sigma2(k, m));
                const float ua = U[k][m] * is * is;
#pragma unroll
                for (int n = 0; n < N; ++n) {
                    an[k][n] = fmaf(lam[n][m], ua, an[k][n]);
                    bn[k][n] = fmaf(lam[n][m], is, bn[k][n]);
                }
            }
        }
        for (int k0 = 0; k0 < K; k0 += KC) {
            float nd[2 * KC * N];
#pragma unroll
            for (int e = 0; e < 2 * KC * N; ++e) nd[e] = 0.0f;
            // bins past T have an = bn = 0 and read frame T - 1; bases past K
            // read base K - 1 and add zero: no branch splits the loads
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const int t = tid + k * nthr;
                const float *vt = a.va + (t < T ? t : T - 1);
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    const bool okc = k0 + c < K;
                    const int kc = okc ? k0 + c : K - 1;
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        const float vl = vt[static_cast<size_t>(kc * N + n) * T];
                        const float vv = okc ? vl : 0.0f;
                        nd[c * N + n] = fmaf(vv, an[k][n], nd[c * N + n]);
                        nd[KC * N + c * N + n] = fmaf(vv, bn[k][n], nd[KC * N + c * N + n]);
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < 2 * KC * N; ++e) nd[e] = wave_sum_last(nd[e]);
            if (lane == 63) {
#pragma unroll
                for (int e = 0; e < 2 * KC * N; ++e) sm.redc[buf][e][wid] = nd[e];
            }
            __syncthreads();
            if (wid == 0) {
                for (int q = lane; q < 2 * KC * N; q += 64) sm.sums[q] = sum_slots<NWS>(sm.redc[buf][q]);
                __threadfence_block();
                __builtin_amdgcn_wave_barrier();
                if (lane < KC * N && k0 + lane / N < K) {
                    const int q = (k0 + lane / N) * N + lane % N;
                    const float tn = sm.t[q] * sqrtf(sm.sums[lane] / sm.sums[KC * N + lane]);
                    if (!(tn > 0.0f) || !(tn < INFINITY)) sm.flag = ST_NONFINITE;
                    sm.t[q] = tn;
                }
            }
            buf ^= 1;
        }
    }
    __syncthreads();
    if (!good || sm.flag != ST_OK) {
        if (tid == 0) a.status[i] = ST_NONFINITE;
        retire();
        return;
    }

    // ---- V-rule terms with the new Lambda_i and t_i
    make_h();
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int t = tid + k * nthr;
        float g[N], e[N];
#pragma unroll
        for (int n = 0; n < N; ++n) g[n] = e[n] = 0.0f;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float is = rcp(sigma2(k, m));
            const float ua = U[k][m] * is * is;
#pragma unroll
            for (int n = 0; n < N; ++n) {
                g[n] = fmaf(lam[n][m], ua, g[n]);
                e[n] = fmaf(lam[n][m], is, e[n]);
            }
        }
        if (t < T) {
#pragma unroll
            for (int n = 0; n < N; ++n) {
                G[t * N + n] = g[n];
                E[t * N + n] = e[n];
            }
        }
    }

    // ---- write back Lambda_i, T_i, W_i
    if (tid == 0) {
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int m = 0; m < M; ++m) a.lam[(static_cast<size_t>(i) * N + n) * M + m] = lam[n][m];
    }
    for (int q = tid; q < K * N; q += nthr) a.tp[static_cast<size_t>(i) * K * N + q] = sm.t[q];
    if (tid < M * M) a.P[static_cast<size_t>(i) * M * M + tid] = sm.Pd[tid];
}

// ------------------------------------------------------------------ V rule
// Partial sums over the frequencies of chunk blockIdx.y for (j, n) =
// divmod(index, N): part[chunk][0][k][index] = sum_i t_ikn G_ijn and
// part[chunk][1][k][index] = sum_i t_ikn E_ijn, each summed over the chunk's
// frequencies in ascending order. The chunk's t is staged in LDS as
// [i][n][k] (zero past the last frequency and past K), so four consecutive
// bases are one 16-byte LDS read; G and E loads are coalesced over the index
// and all in flight before the first FMA.
constexpr int kVThreads = 256;
__global__ void __launch_bounds__(kVThreads) mnmf_v_partial_kernel(const float *G, const float *E, const float *tp,
                                                                   float *part, int F, int T, int N, int K,
                                                                   int fchunk) {
    __shared__ __align__(16) float ts[kMnmfFChunk][kMnmfNMax][kMnmfKMax];
    const int c = blockIdx.y;
    const int i0 = c * fchunk;
    const int ni = min(F, i0 + fchunk) - i0;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int TN = T * N;
    const bool live = idx < TN;
    // the chunk's G and E first, so their latency overlaps the staging of t
    float gs[kMnmfFChunk], es[kMnmfFChunk];
    {
        const float *Gp = G + static_cast<size_t>(i0) * TN + idx;
        const float *Ep = E + static_cast<size_t>(i0) * TN + idx;
#pragma unroll
        for (int ii = 0; ii < kMnmfFChunk; ++ii) {
            gs[ii] = (live && ii < ni) ? Gp[static_cast<size_t>(ii) * TN] : 0.0f;
            es[ii] = (live && ii < ni) ? Ep[static_cast<size_t>(ii) * TN] : 0.0f;
        }
    }
    // every slot of the stage, its loads all issued before the first store
    constexpr int kStage = kMnmfFChunk * kMnmfNMax * kMnmfKMax / kVThreads;
    static_assert(kStage * kVThreads == kMnmfFChunk * kMnmfNMax * kMnmfKMax, "stage tiling");
    float tv[kStage];
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
        const int q = threadIdx.x + r * kVThreads;
        const int ii = q / (kMnmfNMax * kMnmfKMax);
        const int n = (q / kMnmfKMax) % kMnmfNMax;
        const int k = q % kMnmfKMax;
        tv[r] = (ii < ni && n < N && k < K) ? tp[(static_cast<size_t>(i0 + ii) * K + k) * N + n] : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < kStage; ++r) (&ts[0][0][0])[threadIdx.x + r * kVThreads] = tv[r];
    __syncthreads();
    if (!live) return;
    const int n = idx % N;
    float *pn = part + static_cast<size_t>(c) * 2 * K * TN + idx;
    for (int k0 = 0; k0 < K; k0 += 4) {
        float num[4] = {0.f, 0.f, 0.f, 0.f}, den[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ii = 0; ii < kMnmfFChunk; ++ii) {
            const float4 t4 = *reinterpret_cast<const float4 *>(&ts[ii][n][k0]);
            num[0] = fmaf(t4.x, gs[ii], num[0]);
            num[1] = fmaf(t4.y, gs[ii], num[1]);
            num[2] = fmaf(t4.z, gs[ii], num[2]);
            num[3] = fmaf(t4.w, gs[ii], num[3]);
            den[0] = fmaf(t4.x, es[ii], den[0]);
            den[1] = fmaf(t4.y, es[ii], den[1]);
            den[2] = fmaf(t4.z, es[ii], den[2]);
            den[3] = fmaf(t4.w, es[ii], den[3]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (k0 + q < K) {
                pn[static_cast<size_t>(k0 + q) * TN] = num[q];
                pn[static_cast<size_t>(K + k0 + q) * TN] = den[q];
            }
        }
    }
}

// v_jkn <- v_jkn sqrt(num / den), the chunk partials summed in chunk order;
// one thread per (k, index) with index = j N + n, so the partial loads are
// coalesced; activations stored [K][N][T].
__global__ void __launch_bounds__(256) mnmf_v_update_kernel(const float *part, float *va, int nchunk, int T,
                                                            int N, int K, int *flag) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int TN = T * N;
    if (gid >= TN * K) return;
    const int k = gid / TN;
    const int idx = gid - k * TN;
    const int j = idx / N, n = idx - j * N;
    float num = 0.0f, den = 0.0f;
    const float *pc = part + static_cast<size_t>(k) * TN + idx;
    const size_t cs = static_cast<size_t>(2) * K * TN;
    const size_t ds = static_cast<size_t>(K) * TN;
    // up to 32 chunks' loads in flight at once; the zeros past the last
    // chunk leave the sums unchanged
    constexpr int kCB = 32;
    for (int c0 = 0; c0 < nchunk; c0 += kCB) {
        float a[kCB], b[kCB];
#pragma unroll
        for (int q = 0; q < kCB; ++q) {
            const bool ok = c0 + q < nchunk;
            a[q] = ok ? pc[(c0 + q) * cs] : 0.0f;
            b[q] = ok ? pc[(c0 + q) * cs + ds] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < kCB; ++q) {
            num += a[q];
            den += b[q];
        }
    }
    float *v = va + static_cast<size_t>(k * N + n) * T + j;
    const float nv = *v * sqrtf(num / den);
    if (!(nv > 0.0f) || !(nv < INFINITY)) *flag = 1;
    *v = nv;
}

// h_fjn = sum_k t_fkn v_jkn (v stored [K][N][T]) into the frame-model layout [F][T][N], so that
// the likelihood, MWF and parameter calls of the frame model apply.
__global__ void mnmf_h_kernel(const float *tp, const float *va, float *h, int F, int T, int N, int K) {
    const size_t idx = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t total = static_cast<size_t>(F) * T * N;
    if (idx >= total) return;
    const int n = static_cast<int>(idx % N);
    const size_t ft = idx / N;
    const int j = static_cast<int>(ft % T);
    const int f = static_cast<int>(ft / T);
    float s = 0.0f;
    for (int k = 0; k < K; ++k)
        s = fmaf(tp[(static_cast<size_t>(f) * K + k) * N + n], va[static_cast<size_t>(k * N + n) * T + j], s);
    h[idx] = s;
}

// out[c][r] = in[r][c] for an R x C matrix (activation layout changes).
__global__ void transpose_kernel(const float *in, float *out, int R, int C) {
    const size_t idx = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<size_t>(R) * C) return;
    const int r = static_cast<int>(idx / C), c = static_cast<int>(idx % C);
    out[static_cast<size_t>(c) * R + r] = in[idx];
}

// ------------------------------------------------------------------ dispatch
using MnmfFn = void (*)(MnmfLaunch);

template <int M, int N>
static MnmfFn mnmf_bpt(int bpt) {
    switch (bpt) {
        case 4: return mnmf_freq_kernel<M, N, 4>;
        case 8: return mnmf_freq_kernel<M, N, 8>;
        default: return nullptr;
    }
}

#define FFCA_MNMF_N(M)                      \
    switch (N) {                            \
        case 2: return mnmf_bpt<M, 2>(bpt); \
        case 3: return mnmf_bpt<M, 3>(bpt); \
        case 4: return mnmf_bpt<M, 4>(bpt); \
        case 5: return mnmf_bpt<M, 5>(bpt); \
        case 6: return mnmf_bpt<M, 6>(bpt); \
        default: return nullptr;            \
    }

static MnmfFn mnmf_lookup(int M, int N, int bpt) {
    switch (M) {
        case 2: FFCA_MNMF_N(2)
        case 3: FFCA_MNMF_N(3)
        case 4: FFCA_MNMF_N(4)
        default: return nullptr;
    }
}

bool mnmf_supported(int M, int N, int bpt) { return mnmf_lookup(M, N, bpt) != nullptr; }

hipError_t launch_mnmf_freq(int M, int N, int bpt, int threads, const MnmfLaunch &a, hipStream_t s) {
    MnmfFn fn = mnmf_lookup(M, N, bpt);
    if (!fn || threads < 64 || (threads & 63) || threads * bpt > kResidentBins || threads * bpt < a.T ||
        a.K < 1 || a.K > kMnmfKMax)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(a.F), dim3(threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mnmf_v(const float *G, const float *E, const float *tp, float *part, float *va, int F, int T,
                         int N, int K, int fchunk, int *flag, hipStream_t s) {
    if (K < 1 || K > kMnmfKMax || fchunk < 1) return hipErrorInvalidValue;
    const int nchunk = (F + fchunk - 1) / fchunk;
    const int TN = T * N;
    if (fchunk > kMnmfFChunk || N > kMnmfNMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mnmf_v_partial_kernel, dim3((TN + kVThreads - 1) / kVThreads, nchunk), dim3(kVThreads), 0, s,
                       G, E, tp, part, F, T, N, K, fchunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mnmf_v_update_kernel, dim3((TN * K + 255) / 256), dim3(256), 0, s, part, va, nchunk, T, N,
                       K, flag);
    return hipGetLastError();
}

hipError_t launch_transpose(const float *in, float *out, int R, int C, hipStream_t s) {
    const size_t total = static_cast<size_t>(R) * C;
    hipLaunchKernelGGL(transpose_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, in, out,
                       R, C);
    return hipGetLastError();
}

hipError_t launch_mnmf_h(const float *tp, const float *va, float *h, int F, int T, int N, int K, hipStream_t s) {
    const size_t total = static_cast<size_t>(F) * T * N;
    hipLaunchKernelGGL(mnmf_h_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, tp, va, h,
                       F, T, N, K);
    return hipGetLastError();
}

}  // namespace ffca
