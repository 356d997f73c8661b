// FastFCA IP+EM iteration (Algorithm 1, Sec. IV-E) for gfx950.
//
// One workgroup owns one frequency of one mixture (every frequency is an
// independent problem, Sec. II) and runs all requested iterations with the
// frequency's state on chip:
//   registers : x_t (M complex), h_t (N reals), U_t (M reals) for the
//               bins this thread owns (t = tid + k * blockDim, k < BPT)
//   LDS       : P in double precision, its single precision copy, reduction
//               partials
//   wave 0    : the double precision IP sweep (eq:ip1, eq:ip2) and ln|det P|^2
//   wave 1    : meanwhile, the log-likelihood of the previous iterate
// so HBM is touched once per call (read x, h, L, P; write h, L, P). Every
// T-reduction is a fixed-order wavefront DPP tree followed by a fixed-order
// sum over waves, so results are bitwise reproducible for a given launch
// configuration.
//
// Per iteration (N + 2 workgroup barriers):
//   A  sigma^2 = L H (eq:sigmadef), 1/sigma^2, and the M weighted
//      covariances Q_m (eq:wsampcov) accumulated as the M*M real parameters of
//      each Hermitian matrix; the same pass adds the log-likelihood terms of
//      the previous iterate (eq:negll) using its U.
//   IP wave 0: Q_m to double, sweep m = 1..M (eq:ip1, eq:ip2), ln|det P|^2.
//   B  U_mt = |w_m^H x_t|^2 (eq:Udef).
//   C  for n = 1..N in order: posterior gain and power (G_n, Phi_n), the
//      T-reduction giving L[:,n] (with the old H[n,:]), then H[n,:] from the
//      new L[:,n].
#pragma once

#include "device.hpp"
#include "internal.hpp"
#include "ip_sm.hpp"

namespace ffca {

constexpr int kMaxWaves = 16;       // 1024 threads
constexpr int kMaxM = 4;            // resident family: M <= 4
constexpr int kRedW = kMaxM * kMaxM * kMaxM;  // widest reduction (all Q_m, M = 4)
constexpr double kLnPi = 1.1447298858494002;  // ln(pi)

// Reduction slots per workgroup of a launch with BPT bins per thread: one
// per wave of the largest workgroup it allows, at least 4.
constexpr int wave_slots(int bpt) { return kResidentBins / bpt / 64 < 4 ? 4 : kResidentBins / bpt / 64; }

// LDS of one workgroup. Phase A leaves one double precision partial per wave
// of each of the M^3 parameters of the Q_m in redq and one partial per 16-lane
// row (four per wave) of the likelihood terms in red_d; each L reduction of phase C (M
// values, or the 2NM sums of the multiplicative rule) one partial per wave in
// redc, double buffered so that one barrier per reduction suffices. Slots of
// waves that do not exist stay zero. RQ >= M^3, RC >= 2NM values; NWS wave
// slots.
template <int RQ, int RC, int NWS>
struct EmSmem {
    static constexpr int kRowSlots = 4 * NWS;
    static constexpr int kWaveSlots = NWS;
    alignas(16) double redq[RQ][NWS];
    alignas(16) double red_d[4 * NWS];
    alignas(16) float redc[2][RC][NWS];
    double qtot[RQ];
    double2 Pd[kMaxM * kMaxM];
    float2 P32[kMaxM * kMaxM];
    IpSmLds<kMaxM> ip;           // IP scratch (M = 3, 4)
    double ldet[2];              // ln|det P|^2 (|det P|^2 for M = 2) of the IP of iterations of each parity
    int flag;                    // IP status
    int flag_ll;                 // likelihood status
};

// Fixed-order sum of the NS partials of one value, loaded in chunks of up to
// 32 slots whose loads are all issued before the first add.
template <int NS>
__device__ __forceinline__ float sum_slots(const float *p) {
    static_assert(NS % 4 == 0, "slots come in fours");
    constexpr int C = NS < 32 ? NS / 4 : 8;
    float tot = 0.0f;
#pragma unroll
    for (int c0 = 0; c0 < NS / 4; c0 += C) {
        float s[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const float4 a = *reinterpret_cast<const float4 *>(p + 4 * (c0 + i));
            s[i] = (a.x + a.y) + (a.z + a.w);
        }
#pragma unroll
        for (int h = 1; h < C; h *= 2)
#pragma unroll
            for (int i = 0; i + h < C; i += 2 * h) s[i] += s[i + h];
        tot = c0 == 0 ? s[0] : tot + s[0];
    }
    return tot;
}
template <int NS>
__device__ __forceinline__ double sum_slots(const double *p) {
    constexpr int C = NS < 32 ? NS / 4 : 8;
    double tot = 0.0;
#pragma unroll
    for (int c0 = 0; c0 < NS / 4; c0 += C) {
        double s[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const double2 a = *reinterpret_cast<const double2 *>(p + 4 * (c0 + i));
            const double2 b = *reinterpret_cast<const double2 *>(p + 4 * (c0 + i) + 2);
            s[i] = (a.x + a.y) + (b.x + b.y);
        }
#pragma unroll
        for (int h = 1; h < C; h *= 2)
#pragma unroll
            for (int i = 0; i + h < C; i += 2 * h) s[i] += s[i + h];
        tot = c0 == 0 ? s[0] : tot + s[0];
    }
    return tot;
}

// The same fixed-order sums over the populated slots only: the partials of
// nw waves fill the first 4 nw row slots (first nw wave slots). Slots are
// summed in groups of four waves (16 row slots, 4 wave slots), each group as
// a tree and the groups in order; the slots past the last wave hold zeros.
template <int NS>
__device__ __forceinline__ float sum_rows(const float *p, int nw) {
    float tot = 0.0f;
#pragma unroll
    for (int g = 0; g < NS / 16; ++g) {
        if (g == 0 || g * 4 < nw) {
            float s[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 a = *reinterpret_cast<const float4 *>(p + 16 * g + 4 * i);
                s[i] = (a.x + a.y) + (a.z + a.w);
            }
            const float u = (s[0] + s[1]) + (s[2] + s[3]);
            tot = g == 0 ? u : tot + u;
        }
    }
    return tot;
}
template <int NS>
__device__ __forceinline__ double sum_rows(const double *p, int nw) {
    double tot = 0.0;
#pragma unroll
    for (int g = 0; g < NS / 16; ++g) {
        if (g == 0 || g * 4 < nw) {
            double s[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double2 a = *reinterpret_cast<const double2 *>(p + 16 * g + 2 * i);
                s[i] = a.x + a.y;
            }
            const double u = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
            tot = g == 0 ? u : tot + u;
        }
    }
    return tot;
}
template <int NS>
__device__ __forceinline__ float sum_waves(const float *p, int nw) {
    float tot = 0.0f;
#pragma unroll
    for (int g = 0; g < NS / 4; ++g) {
        if (g == 0 || g * 4 < nw) {
            const float4 a = *reinterpret_cast<const float4 *>(p + 4 * g);
            const float u = (a.x + a.y) + (a.z + a.w);
            tot = g == 0 ? u : tot + u;
        }
    }
    return tot;
}
template <int NS>
__device__ __forceinline__ double sum_waves(const double *p, int nw) {
    double tot = 0.0;
#pragma unroll
    for (int g = 0; g < NS / 4; ++g) {
        if (g == 0 || g * 4 < nw) {
            const double2 a = *reinterpret_cast<const double2 *>(p + 4 * g);
            const double2 b = *reinterpret_cast<const double2 *>(p + 4 * g + 2);
            const double u = (a.x + a.y) + (b.x + b.y);
            tot = g == 0 ? u : tot + u;
        }
    }
    return tot;
}

// IP sweep for M = 2 in registers (every lane of wave 0 computes the same
// values). For 2 x 2 matrices the solve of eq:ip1, w = (P^H Q_m)^{-1} e_m,
// equals Q_m^{-1} P^{-H} e_m, and both inverses are adjugates over
// determinants:
//   P^{-H} e_m = b / conj(d),  d = det P,  b = conj(P11, -P01) (m = 1) or
//                                          conj(-P10, P00) (m = 2);
//   Q^{-1} = adj(Q) / det Q.
// With u = adj(Q) b and s = b^H u, eq:ip2's normalization w^H Q w = 1 makes
//   w = u d / sqrt(s det(Q) |d|^2),
// one reciprocal square root per column and no division. The second column
// does not wait for the first one's normalization: with the new first column
// w_1 = c u_1 (c = d / sqrt(s_1 det(Q_1) |d|^2)), the second column's b is
// conj(c) beta, beta = conj(-u_1[1], u_1[0]), and the new determinant is
// c delta, delta = u_1[0] P11 - P01 u_1[1], so that
//   w_2 = nu delta / sqrt(sigma det(Q_2) |delta|^2),
//   nu = adj(Q_2) beta, sigma = beta^H nu,
// in which c cancels. The system is taken as singular when
// |det(P^H Q)|^2 = |d|^2 det(Q)^2 falls below tol^2 (|P|_F^2 |Q|_F^2)^2, the
// fourth power of a bound on its largest entry, with P the matrix each
// column's solve sees.
// q: the 8 Hermitian parameters (Q_1 then Q_2) of T Q_m, the sums before
// the division by T; qscale = sqrt(T). Scaling Q by T scales u and s by T and
// det Q by T^2, so w of the scaled sums is w / sqrt(T), and the pivot test
// is scale free: one multiplication per column replaces eight scalings.
// The checks are folded into one status without branches; nothing is
// stored unless both columns pass.
// P: the current P (row-major), read by the caller before the slot sums so
// that both LDS reads are in flight together.
// det2: |det P|^2 of the new P (its logarithm is left to the caller, off the
// IP's critical path).
template <class Smem>
__device__ __forceinline__ int ip_sweep_reg2(Smem &sm, const cd (&P)[4], const double (&q)[8], double qscale,
                                             double &det2) {
    const cd P00 = P[0], P01 = P[1], P10 = P[2], P11 = P[3];
    // the Q_m terms of both columns
    double dq[2], nq[2];
    bool fin[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const double q00 = q[4 * m + 0], q11 = q[4 * m + 1];
        const cd q01 = cmk(q[4 * m + 2], q[4 * m + 3]);
        fin[m] = (fabs(q00) < INFINITY) && (fabs(q11) < INFINITY) && (abs2(q01) < INFINITY);
        dq[m] = q00 * q11 - abs2(q01);
        nq[m] = q00 * q00 + q11 * q11 + 2.0 * abs2(q01);
    }
    auto adjq = [&](int m, cd b0, cd b1, cd &u0, cd &u1) {
        const double q00 = q[4 * m + 0], q11 = q[4 * m + 1];
        const cd q01 = cmk(q[4 * m + 2], q[4 * m + 3]);
        u0 = q11 * b0 - q01 * b1;
        u1 = q00 * b1 - conjd(q01) * b0;
    };
    auto pivot_ok = [&](int m, double d2, double np, double t) {
        return (d2 * dq[m] * dq[m] >= kPivotTol * kPivotTol * (np * nq[m]) * (np * nq[m])) && (t > 0.0) &&
               (t < INFINITY);
    };
    // first column
    cd a0, a1;
    adjq(0, conjd(P11), cmk(-P01.re, P01.im), a0, a1);
    const double sb = (P11 * a0 - P01 * a1).re;  // b^H u with b = conj(P11, -P01)
    const cd d = P00 * P11 - P01 * P10;
    const double d2 = abs2(d);
    const double np = (abs2(P00) + abs2(P01)) + (abs2(P10) + abs2(P11));
    const double t = sb * dq[0] * d2;
    // second column from u of the first: beta = conj(-a1, a0)
    cd n0, n1;
    const cd be0 = cmk(-a1.re, a1.im), be1 = conjd(a0);
    adjq(1, be0, be1, n0, n1);
    const double sg = (conjd(be0) * n0 + conjd(be1) * n1).re;
    const cd de = a0 * P11 - P01 * a1;
    const double de2 = abs2(de);
    const double t2 = sg * dq[1] * de2;
    // both normalizations
    const double r = rsqrt_d(t) * qscale;
    const cd c = r * d;
    const cd W00 = a0 * c, W10 = a1 * c;
    const double r2 = rsqrt_d(t2) * qscale;
    const cd W01 = r2 * (n0 * de), W11 = r2 * (n1 * de);
    // the second solve's pivot test on the P it sees: [w_1 | p_2]
    const double c2 = abs2(c);
    const double np2 = c2 * (abs2(a0) + abs2(a1)) + (abs2(P01) + abs2(P11));
    int stat = !fin[0] ? ST_NONFINITE : (!pivot_ok(0, d2, np, t) ? ST_SINGULAR : ST_OK);
    const int stat2 = !fin[1] ? ST_NONFINITE : (!pivot_ok(1, c2 * de2, np2, t2) ? ST_SINGULAR : ST_OK);
    stat = stat != ST_OK ? stat : stat2;
    if (stat != ST_OK) return stat;
    det2 = abs2(W00 * W11 - W01 * W10);
    sm.Pd[0] = st(W00);
    sm.Pd[1] = st(W01);
    sm.Pd[2] = st(W10);
    sm.Pd[3] = st(W11);
    sm.P32[0] = make_float2(static_cast<float>(W00.re), static_cast<float>(W00.im));
    sm.P32[1] = make_float2(static_cast<float>(W01.re), static_cast<float>(W01.im));
    sm.P32[2] = make_float2(static_cast<float>(W10.re), static_cast<float>(W10.im));
    sm.P32[3] = make_float2(static_cast<float>(W11.re), static_cast<float>(W11.im));
    return ST_OK;
}

// COV = false: every bin is one frame and its statistics come from x_t.
// COV = true: every bin is a block of the piecewise stationary model (Sec. VI)
// whose block covariance Xhat_j (M^2 real parameters, read from it.z) replaces
// x_j x_j^H: Q_m takes Xhat_j / sigma^2 and U_mj = w_m^H Xhat_j w_m.
template <int M, int N, int BPT, bool COV, class Smem>
__device__ __forceinline__ void em_item(const WorkItem &it, int n_iter, int algo, double alarm, int trace_off,
                                        Smem &sm) {
    constexpr int NQ = M * M * M;
    constexpr int M2 = M * M;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    constexpr int NR = Smem::kRowSlots;
    constexpr int NW = Smem::kWaveSlots;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const bool row_lead = (lane & 15) == 0;
    const int row_slot = 4 * wid + (lane >> 4);
    const int nw = nthr >> 6;
    const int llw = nw > 1 ? 1 : 0;  // wave that finishes the likelihood while wave 0 runs the IP
    const int T = it.T;
    const float invTf = 1.0f / static_cast<float>(T);
    const double invT = 1.0 / static_cast<double>(T);
    const double sqrtT = sqrt(static_cast<double>(T));

    // ---- load the frequency's state. Bins t >= T hold x = 0 and h = 1: they
    // add nothing to Q or U, and mk = 0 drops them from the other sums.
    float2 xr[BPT][COV ? 1 : M];
    float zr[BPT][COV ? M2 : 1];
    float vr[BPT][N];
    float U[BPT][M];
    float mk[BPT];
    // M = 2 and M = 4 (four bins per thread) keep sigma^2 and 1/sigma^2 of
    // every bin from phase A through phase C: source 1 uses them as they are,
    // and after each later source's update sigma^2 is formed again from L and
    // H (M = 2) or changed by that source's own term (M = 4: two FMAs instead
    // of N; formed again when the change cancels, see below). Phase A
    // recomputes them from L and H every iteration, so rounding does not
    // accumulate across iterations. The other shapes would lose occupancy to
    // the 2 M BPT registers (M = 3 drops from three waves per SIMD to two;
    // M = 2 with eight bins per thread beyond four sources, from two to one).
    constexpr bool kKeep = ((M == 2) && (BPT <= 4 || N <= 4)) || (M == 4 && BPT == 4);
    // a running sigma^2 below this fraction of its previous value has lost
    // more than two bits to cancellation and is formed again (a single
    // precision emulation over twelve decades bounds the per-bin error by
    // 8e-7 with it, 1e-4 with 1/64, and finds 3.6 without it)
    constexpr float kSgDrop = 0.25f;
    float sg[kKeep ? BPT : 1][M];
    float wr[kKeep ? BPT : 1][M];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int t = tid + k * nthr;
        const bool valid = t < T;
        mk[k] = valid ? 1.0f : 0.0f;
        if constexpr (COV) {
#pragma unroll
            for (int e = 0; e < M2; ++e) zr[k][e] = valid ? it.z[t * M2 + e] : 0.0f;
        } else {
#pragma unroll
            for (int r = 0; r < M; ++r) xr[k][r] = valid ? it.x[t * M + r] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int n = 0; n < N; ++n) vr[k][n] = valid ? it.v[t * N + n] : 1.0f;
#pragma unroll
        for (int m = 0; m < M; ++m) U[k][m] = 0.0f;
    }
    float lam[N][M];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int m = 0; m < M; ++m) lam[n][m] = it.lam[n * M + m];
    if (tid < M * M) {
        sm.Pd[tid] = it.P[tid];
    }
    if (tid == 0) {
        sm.flag = ST_OK;
        sm.flag_ll = ST_OK;
    }
    for (int i = tid; i < static_cast<int>(sizeof(sm.redq) / sizeof(double)); i += nthr) (&sm.redq[0][0])[i] = 0.0;
    for (int i = tid; i < static_cast<int>(sizeof(sm.redc) / sizeof(float)); i += nthr) (&sm.redc[0][0][0])[i] = 0.0f;
    for (int i = tid; i < NR; i += nthr) sm.red_d[i] = 0.0;
    __syncthreads();

    double ldet_prev = M == 2 ? 1.0 : 0.0;  // ln|det P|^2 (M = 2: |det P|^2) of the latest iterate (wave 0)
    double *const ll_trace = it.ll_trace + trace_off;
    double ll_last = 0.0;  // LL of the previous iterate (likelihood wave)
    int buf = 0;
    int status = ST_OK;

    for (int iter = 0; iter <= n_iter; ++iter) {
        const bool last = (iter == n_iter);
        if constexpr (!COV && M >= 3) {
            // x x^H is formed again every iteration instead of being kept
            // across iterations: for M >= 3 its M^2 values per bin cost more
            // in occupancy than the 3M^2 operations that recompute them
#pragma unroll
            for (int k = 0; k < BPT; ++k)
#pragma unroll
                for (int r = 0; r < M; ++r) asm volatile("" : "+v"(xr[k][r].x), "+v"(xr[k][r].y));
        }
        // ---------------- phase A: weights, Q_m, LL terms of the previous iterate
        float q[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) q[i] = 0.0f;
        float lg2 = 0.0f;  // sum of log2 sigma^2 over this lane's bins
        float uw = 0.0f;   // sum of U / sigma^2 (zero for bins t >= T)
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            float w[M];
            float s2[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float s = 0.0f;
#pragma unroll
                for (int n = 0; n < N; ++n) s = fmaf(vr[k][n], lam[n][m], s);
                s2[m] = s;
                w[m] = rcp(s);
                if constexpr (kKeep) {
                    sg[k][m] = s;
                    wr[k][m] = w[m];
                }
            }
            if (iter > 0) {
                float l = 0.0f;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    l += log2_fast(s2[m]);
                    uw = fmaf(U[k][m], w[m], uw);
                }
                lg2 = fmaf(mk[k], l, lg2);
            }
            if (!last) {
                // Z_t = x_t x_t^H (or Xhat_j) in Hermitian real parameters
                float z[M * M];
                if constexpr (COV) {
#pragma unroll
                    for (int e = 0; e < M2; ++e) z[e] = zr[k][e];
                } else {
#pragma unroll
                    for (int r = 0; r < M; ++r)
                        z[r] = xr[k][r].x * xr[k][r].x + xr[k][r].y * xr[k][r].y;
                    int p = M;
#pragma unroll
                    for (int r = 0; r < M; ++r)
#pragma unroll
                        for (int c = r + 1; c < M; ++c) {
                            z[p] = xr[k][r].x * xr[k][c].x + xr[k][r].y * xr[k][c].y;
                            z[p + 1] = xr[k][r].y * xr[k][c].x - xr[k][r].x * xr[k][c].y;
                            p += 2;
                        }
                }
#pragma unroll
                for (int m = 0; m < M; ++m)
#pragma unroll
                    for (int e = 0; e < M * M; ++e) q[m * M * M + e] = fmaf(w[m], z[e], q[m * M * M + e]);
            }
        }
        // wave partials of Q (four values per reduction, value 4g + r in row
        // r) and row partials of the LL terms to LDS. Each lane's partial
        // (BPT bins) is single precision; every sum across lanes and waves is
        // double precision: with the single precision tree the rounding of
        // the Q_m, amplified by an ill-conditioned IP system, moved the
        // likelihood by more than 1e-6 nats per bin within ten iterations.
        if (!last) {
            constexpr int NGQ = (NQ + 3) / 4;
            double tq[NGQ];
            wave_sums_rows<NQ>(q, tq);
            if ((lane & 15) == 0) {
#pragma unroll
                for (int g = 0; g < NGQ; ++g)
                    if (4 * g + (lane >> 4) < NQ) sm.redq[4 * g + (lane >> 4)][wid] = tq[g];
            }
        }
        double llp = row_sum(static_cast<double>(lg2) * static_cast<double>(kLn2f) + static_cast<double>(uw));
        if (row_lead) sm.red_d[row_slot] = llp;
        __syncthreads();
        if (wid == llw && iter > 0) {
            // eq:negll for the previous iterate, beside the IP on wave 0
            const double s = sum_rows<NR>(sm.red_d, nw);
            // M = 2: the IP wave left |det P|^2; its logarithm in double
            // precision is taken here, beside the IP of the next iterate
            const double ldp = sm.ldet[(iter - 1) & 1];
            const double ll = (M == 2 ? log(ldp) : ldp) - static_cast<double>(M) * kLnPi - s * invT;
            if (lane == 0) {
                ll_trace[iter - 1] = ll;
                if (!(ll == ll) || ll == INFINITY || ll == -INFINITY)
                    sm.flag_ll = ST_NONFINITE;
                else if (iter > 1 && ll < ll_last - alarm)  // Algorithms 1 and 2 never lower it
                    sm.flag_ll = ST_DECREASE;
            }
            ll_last = ll;
        }
        if (wid == 0 && !last) {
            double ldet = 0.0;
            if constexpr (M == 2) {
                // lane i sums value i % 8 over the row slots, then every lane
                // reads the eight sums of lanes 0-7 from registers
                const cd Pc[4] = {ld(sm.Pd[0]), ld(sm.Pd[1]), ld(sm.Pd[2]), ld(sm.Pd[3])};
                double qs[8];
                const double mine = sum_waves<NW>(sm.redq[lane & 7], nw);
#pragma unroll
                for (int i = 0; i < 8; ++i) qs[i] = readlane_d(mine, i);
                status = ip_sweep_reg2(sm, Pc, qs, sqrtT, ldet);
            } else {
                if (lane < NQ) sm.qtot[lane] = sum_waves<NW>(sm.redq[lane], nw) * invT;
                __threadfence_block();
                __builtin_amdgcn_wave_barrier();
                // IP sweep in double precision through the inverses
                status = ip_sm<M, kMaxM>(sm.qtot, sm.Pd, sm.P32, sm.ip, ldet);
            }
            if (status == ST_OK) {
                ldet_prev = ldet;
                if (lane == 0) sm.ldet[iter & 1] = ldet;
            }
            if (lane == 0) sm.flag = status;
        }
        if (last) break;
        __syncthreads();
        status = sm.flag;
        if (status == ST_OK) status = sm.flag_ll;
        if (status != ST_OK) break;

        // ---------------- phase B: U = |P^H x|^2, or w_m^H Xhat w_m
        if constexpr (COV) {
            // U_m = sum_e c_m[e] z[e]: |P_rm|^2 on the diagonal parameters,
            // 2 Re and -2 Im of conj(P_rm) P_cm on those of entry (r, c), r < c
            float cm[M][M2];
#pragma unroll
            for (int m = 0; m < M; ++m) {
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    const float2 a = sm.P32[r * M + m];
                    cm[m][r] = a.x * a.x + a.y * a.y;
                }
                int p = M;
#pragma unroll
                for (int r = 0; r < M; ++r)
#pragma unroll
                    for (int c = r + 1; c < M; ++c) {
                        const float2 a = sm.P32[r * M + m], b = sm.P32[c * M + m];
                        cm[m][p] = 2.0f * (a.x * b.x + a.y * b.y);
                        cm[m][p + 1] = -2.0f * (a.x * b.y - a.y * b.x);
                        p += 2;
                    }
            }
#pragma unroll
            for (int k = 0; k < BPT; ++k)
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    float u = 0.0f;
#pragma unroll
                    for (int e = 0; e < M2; ++e) u = fmaf(cm[m][e], zr[k][e], u);
                    U[k][m] = fmaxf(u, 0.0f);
                }
        } else {
            float2 Pw[M][M];
#pragma unroll
            for (int i = 0; i < M * M; ++i) Pw[i / M][i % M] = sm.P32[i];
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    float yr = 0.0f, yi = 0.0f;
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        // conj(P[r][m]) * x_r
                        yr = fmaf(Pw[r][m].x, xr[k][r].x, yr);
                        yr = fmaf(Pw[r][m].y, xr[k][r].y, yr);
                        yi = fmaf(Pw[r][m].x, xr[k][r].y, yi);
                        yi = fmaf(-Pw[r][m].y, xr[k][r].x, yi);
                    }
                    U[k][m] = yr * yr + yi * yi;
                }
            }
        }

        // ---------------- phase C (Algorithm 2): MM update of L, then of H
        if (algo == kAlgoMM) {
            // numerators / denominators of the L rule: sum_t U v / sigma^4, sum_t v / sigma^2
            float nd[2 * N * M];
#pragma unroll
            for (int i = 0; i < 2 * N * M; ++i) nd[i] = 0.0f;
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    float s = 0.0f;
#pragma unroll
                    for (int nn = 0; nn < N; ++nn) s = fmaf(vr[k][nn], lam[nn][m], s);
                    const float is = mk[k] * rcp(s);
                    const float ua = U[k][m] * is * is;
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        nd[n * M + m] = fmaf(ua, vr[k][n], nd[n * M + m]);
                        nd[N * M + n * M + m] = fmaf(is, vr[k][n], nd[N * M + n * M + m]);
                    }
                }
            }
            constexpr int NG = (2 * N * M + 3) / 4;
            float tot[NG];
            wave_sums_rows<2 * N * M>(nd, tot);
            if ((lane & 15) == 0) {
#pragma unroll
                for (int g = 0; g < NG; ++g)
                    if (4 * g + (lane >> 4) < 2 * N * M) sm.redc[buf][4 * g + (lane >> 4)][wid] = tot[g];
            }
            __syncthreads();
            const float mine = lane < 2 * N * M ? sum_waves<NW>(sm.redc[buf][lane], nw) : 0.0f;
            bool good = true;
#pragma unroll
            for (int n = 0; n < N; ++n)
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const float num = readlane_f(mine, n * M + m);
                    const float den = readlane_f(mine, N * M + n * M + m);
                    const float l = lam[n][m] * sqrtf(num / den);
                    good = good && (l > 0.0f) && (l < INFINITY);
                    lam[n][m] = l;
                }
            buf ^= 1;
            if (!good) {
                status = ST_NONFINITE;
                break;
            }
            // H rule with the new L (local to each bin)
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                float num[N], den[N];
#pragma unroll
                for (int n = 0; n < N; ++n) num[n] = den[n] = 0.0f;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    float s = 0.0f;
#pragma unroll
                    for (int nn = 0; nn < N; ++nn) s = fmaf(vr[k][nn], lam[nn][m], s);
                    const float is = rcp(s);
                    const float ua = U[k][m] * is * is;
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        num[n] = fmaf(lam[n][m], ua, num[n]);
                        den[n] = fmaf(lam[n][m], is, den[n]);
                    }
                }
#pragma unroll
                for (int n = 0; n < N; ++n) vr[k][n] = mk[k] != 0.0f ? vr[k][n] * sqrtf(num[n] / den[n]) : 1.0f;
            }
            continue;
        }

        // ---------------- phase C (Algorithm 1): EM over sources, in order.
        // With g = h l / sigma^2 the posterior power of eq:Phidef divided by h is
        //   e = l (1 + g (U / sigma^2 - 1)),
        // so the L update is the T-mean of e and the H update is
        //   h <- h * (1/M) sum_m e_m / l_new,m,
        // which needs no reciprocal of h.
        // a non-positive or non-finite L is recorded and acted on after the
        // last source, so no branch waits on the check inside the loop (the
        // failing frequency's state is left as it is then)
        bool bad = false;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            float part[M];
            float e[BPT][M];
            float l2[M];
            float lold[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                part[m] = 0.0f;
                l2[m] = lam[n][m] * lam[n][m];
                lold[m] = lam[n][m];
            }
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    float w;
                    if constexpr (kKeep) {
                        w = wr[k][m];
                    } else {
                        float s = 0.0f;
#pragma unroll
                        for (int nn = 0; nn < N; ++nn) s = fmaf(vr[k][nn], lam[nn][m], s);
                        w = rcp(s);
                    }
                    const float r = fmaf(U[k][m], w, -1.0f);
                    const float gl = (vr[k][n] * w) * l2[m];
                    const float ek = fmaf(gl, r, lam[n][m]);
                    e[k][m] = ek;
                    part[m] = fmaf(mk[k], ek, part[m]);
                }
            }
            float tot[1];
            wave_sums_rows<M>(part, tot);
            if ((lane & 15) == 0 && (lane >> 4) < M) sm.redc[buf][lane >> 4][wid] = tot[0];
            __syncthreads();
            // every lane sums the same slots in the same order, so L stays
            // uniform without cross-lane moves
            float c[M];
            bool good = true;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const float l = sum_waves<NW>(sm.redc[buf][m], nw) * invTf;
                good = good && (l > 0.0f) && (l < INFINITY);
                lam[n][m] = l;
                c[m] = rcp(l * static_cast<float>(M));
            }
            buf ^= 1;
            bad = bad || !good;
            bool drop = false;  // some bin's sigma^2 fell below kSgDrop of its value
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                float s = 0.0f;
#pragma unroll
                for (int m = 0; m < M; ++m) s = fmaf(e[k][m], c[m], s);
                const float vold = vr[k][n];
                const float vnew = mk[k] != 0.0f ? vold * s : 1.0f;
                vr[k][n] = vnew;
                if constexpr (kKeep) {
                    if (n + 1 < N) {
#pragma unroll
                        for (int m = 0; m < M; ++m) {
                            if constexpr (M == 2) {
                                // two channels: the sum itself costs one FMA more
                                float t = 0.0f;
#pragma unroll
                                for (int nn = 0; nn < N; ++nn) t = fmaf(vr[k][nn], lam[nn][m], t);
                                sg[k][m] = t;
                            } else {
                                const float sn = fmaf(lam[n][m], vnew, fmaf(-lold[m], vold, sg[k][m]));
                                drop = drop || !(sn >= kSgDrop * sg[k][m]);
                                sg[k][m] = sn;
                            }
                        }
                    }
                }
            }
            if constexpr (kKeep) {
                if (n + 1 < N) {
                    // Where the updated source dominated a bin and its term
                    // collapsed, the subtraction above cancels most digits of
                    // sigma^2; then (rarely) the whole wavefront forms the sums
                    // again from L and H.
                    if (M != 2 && __any(drop)) {
#pragma unroll
                        for (int k = 0; k < BPT; ++k)
#pragma unroll
                            for (int m = 0; m < M; ++m) {
                                float t = 0.0f;
#pragma unroll
                                for (int nn = 0; nn < N; ++nn) t = fmaf(vr[k][nn], lam[nn][m], t);
                                sg[k][m] = t;
                            }
                    }
#pragma unroll
                    for (int k = 0; k < BPT; ++k)
#pragma unroll
                        for (int m = 0; m < M; ++m) wr[k][m] = rcp(sg[k][m]);
                }
            }
        }
        if (bad) status = ST_NONFINITE;
        if (status != ST_OK) break;
    }

    // the likelihood wave's verdict on the last iterate
    __syncthreads();
    if (status == ST_OK) status = sm.flag_ll;

    // ---- write back the state
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int t = tid + k * nthr;
        if (t < T) {
#pragma unroll
            for (int n = 0; n < N; ++n) it.v[t * N + n] = vr[k][n];
        }
    }
    if (tid == 0) {
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int m = 0; m < M; ++m) it.lam[n * M + m] = lam[n][m];
    }
    if (wid == 0) {
        if (lane < M * M) it.P[lane] = sm.Pd[lane];
        if (lane == 0) {
            *it.ldet = (M == 2) ? log(ldet_prev) : ldet_prev;
            if (status != ST_OK) *it.status = status;
        }
    }
    __syncthreads();  // the LDS is reused by the next item of a persistent launch
}

}  // namespace ffca
