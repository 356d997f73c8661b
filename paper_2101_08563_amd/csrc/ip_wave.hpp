// Lane-parallel double precision IP sweep shared by the IP+EM kernels.
#pragma once

#include "device.hpp"
#include "internal.hpp"

namespace ffca {

__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Index (r, c), r < c, of the p-th strictly upper entry in row-major order.
template <int M>
__device__ __forceinline__ void upper_pair(int p, int &r, int &c) {
    r = 0;
    int rowlen = M - 1;
    while (p >= rowlen) {
        p -= rowlen;
        ++r;
        --rowlen;
    }
    c = r + 1 + p;
}
template <int M>
__device__ __forceinline__ int upper_index(int r, int c) {  // r < c
    return r * (2 * M - r - 1) / 2 + (c - r - 1);
}

// LDS work space of the lane-parallel IP sweep for M <= MM.
template <int MM>
struct IpLds {
    double2 Qd[MM * MM * MM];   // the M weighted covariances as full matrices
    double2 A[MM * (MM + 1)];   // augmented system [P^H Q_m | e_m]
};

// Lane-parallel IP sweep on one wavefront (all 64 lanes call it), one
// matrix element per lane. qtot: the M weighted covariances Q_m (eq:wsampcov)
// as Hermitian real parameters (M diagonal entries, then re/im of the upper
// triangle), already divided by T. For m = 1..M in order: A = P^H Q_m,
// Gauss-Jordan elimination with partial pivoting on [A | e_m] (eq:ip1),
// w_m <- w_m / sqrt(w_m^H Q_m w_m) (eq:ip2); then ln|det P|^2. P (double, Pd)
// is updated in place and copied to P32. The wavefront executes its LDS
// instructions in order, so no barrier is needed between the phases.
//
// Each elimination step is two LDS round trips: every lane reads column k to
// find the pivot row p, then reads the four entries it needs of the matrix
// before the step (its own entry and column-k entry in its source row, the
// pivot row's entry in its column and the pivot) and writes its entry of the
// matrix after the swap of rows k and p and the elimination. All reads of a
// step are issued before its writes, which the in-order LDS makes safe.
template <int M, int MM>
__device__ __noinline__ int ip_wave(const double *qtot, double2 *Pd, float2 *P32, IpLds<MM> &w,
                                    double &ldet) {
    constexpr int M2 = M * M;
    constexpr int W = M + 1;              // row stride of the augmented matrix
    constexpr int NE = M * W;             // entries of [A | e_m]
    constexpr int NS = (NE + 63) / 64;    // entries per lane
    const int lane = threadIdx.x & 63;
    const bool el = lane < M2;
    const int r = lane / M, c = lane % M;
    bool finite = true;
    for (int i = lane; i < M * M2; i += 64) {
        const int m = i / M2, rr = (i / M) % M, cc = i % M;
        const double *q = qtot + m * M2;
        double2 v;
        if (rr == cc) {
            v = make_double2(q[rr], 0.0);
        } else {
            const int lo = rr < cc ? rr : cc, hi = rr < cc ? cc : rr;
            const int p = upper_index<M>(lo, hi);
            const double re = q[M + 2 * p], im = q[M + 2 * p + 1];
            v = make_double2(re, rr < cc ? im : -im);
        }
        finite = finite && fabs(v.x) < INFINITY && fabs(v.y) < INFINITY;
        w.Qd[i] = v;
    }
    if (__any(!finite)) return ST_NONFINITE;
#pragma unroll 1
    for (int m = 0; m < M; ++m) {
        double a2 = 0.0;
        if (el) {
            cd s = cmk(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < M; ++k) s = s + conjd(ld(Pd[k * M + r])) * ld(w.Qd[m * M2 + k * M + c]);
            w.A[r * W + c] = st(s);
            a2 = abs2(s);
        }
        if (lane < M) w.A[lane * W + M] = make_double2(lane == m ? 1.0 : 0.0, 0.0);
        const double amax2 = wave_max(a2);
        if (!(amax2 > 0.0) || !(amax2 < INFINITY)) return ST_SINGULAR;
        // one elimination step; the loop over k is unrolled except for M = 3,
        // whose kernels would lose their third wave per SIMD to the registers
        bool sing = false;
        auto step = [&](int k) {
            // the whole column in one round trip (rows above k are read and ignored)
            double colv[M];
#pragma unroll
            for (int i = 0; i < M; ++i) colv[i] = abs2(ld(w.A[i * W + k]));
            int p = k;
            double best = 0.0;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (i == k) best = colv[i];
                if (i > k && colv[i] > best) {
                    best = colv[i];
                    p = i;
                }
            }
            if (!(best >= kPivotTol * kPivotTol * amax2)) {
                sing = true;
                return;
            }
            cd nv[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int e = lane + 64 * q;
                const int i = e / W, j = e - (e / W) * W;
                const int src = i == k ? p : (i == p ? k : i);
                // lanes past the matrix read a valid entry and store nothing
                const int si = e < NE ? src : 0, sj = e < NE ? j : 0;
                const cd arow = ld(w.A[si * W + sj]);
                const cd acol = ld(w.A[si * W + k]);
                const cd prow = ld(w.A[p * W + sj]);
                const cd piv = ld(w.A[p * W + k]);
                const cd ipiv = rcp_d(abs2(piv)) * conjd(piv);
                const cd pr = prow * ipiv;
                nv[q] = i == k ? pr : arow - acol * pr;
            }
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int e = lane + 64 * q;
                if (e < NE) w.A[e] = st(nv[q]);
            }
        };
        if constexpr (M == 3) {
#pragma unroll 1
            for (int k = 0; k < M && !sing; ++k) step(k);
        } else {
#pragma unroll
            for (int k = 0; k < M; ++k)
                if (!sing) step(k);
        }
        if (sing) return ST_SINGULAR;
        // w = last column; normalize so that w^H Q_m w = 1
        double qt = 0.0;
        if (el) {
            const cd wr = ld(w.A[r * W + M]), wc = ld(w.A[c * W + M]);
            qt = (conjd(wr) * ld(w.Qd[m * M2 + r * M + c]) * wc).re;
        }
        const double qq = wave_sum(qt);
        if (!(qq > 0.0) || !(qq < INFINITY)) return ST_SINGULAR;
        const double inv = rsqrt_d(qq);
        if (lane < M) Pd[lane * M + m] = st(inv * ld(w.A[lane * W + M]));
    }
    // ln|det P|^2: elimination with partial pivoting on a copy of P (row
    // stride W), the product of the squared pivot moduli kept as a mantissa
    // and a binary exponent, one logarithm at the end
    if (el) w.A[r * W + c] = Pd[lane];
    double mant = 1.0;
    int ex = 0;
    bool sing = false;
    auto dstep = [&](int k) {
        double colv[M];
#pragma unroll
        for (int i = 0; i < M; ++i) colv[i] = abs2(ld(w.A[i * W + k]));
        int p = k;
        double best = 0.0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (i == k) best = colv[i];
            if (i > k && colv[i] > best) {
                best = colv[i];
                p = i;
            }
        }
        if (!(best > 0.0) || !(best < INFINITY)) {
            sing = true;
            return;
        }
        int e2;
        mant = frexp(mant * best, &e2);
        ex += e2;
        if (k + 1 < M) {
            const int i = r, j = c;
            const int src = i == k ? p : (i == p ? k : i);
            const int si = el ? src : 0, sj = el ? j : 0;
            const cd arow = ld(w.A[si * W + sj]);
            const cd acol = ld(w.A[si * W + k]);
            const cd prow = ld(w.A[p * W + sj]);
            const cd piv = ld(w.A[p * W + k]);
            const cd ipiv = rcp_d(abs2(piv)) * conjd(piv);
            const cd nv = i == k ? prow : (i > k ? arow - acol * (prow * ipiv) : arow);
            if (el) w.A[i * W + j] = st(nv);
        }
    };
    if constexpr (M == 3) {
#pragma unroll 1
        for (int k = 0; k < M && !sing; ++k) dstep(k);
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k)
            if (!sing) dstep(k);
    }
    if (sing) return ST_SINGULAR;
    ldet = log(mant) + static_cast<double>(ex) * 0.69314718055994531;
    if (el) {
        const double2 pv = Pd[lane];
        P32[lane] = make_float2(static_cast<float>(pv.x), static_cast<float>(pv.y));
    }
    return ST_OK;
}

}  // namespace ffca
