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
    double2 colk[MM];           // elimination factors of the current column
};

// Lane-parallel IP sweep on one wavefront (all 64 lanes call it), one
// matrix element per lane. qtot: the M weighted covariances Q_m (eq:wsampcov)
// as Hermitian real parameters (M diagonal entries, then re/im of the upper
// triangle), already divided by T. For m = 1..M in order: A = P^H Q_m,
// Gauss-Jordan elimination with partial pivoting on [A | e_m] (eq:ip1),
// w_m <- w_m / sqrt(w_m^H Q_m w_m) (eq:ip2); then ln|det P|^2. P (double, Pd)
// is updated in place and copied to P32. The wavefront executes its LDS
// instructions in order, so no barrier is needed between the phases.
template <int M, int MM>
__device__ __noinline__ int ip_wave(const double *qtot, double2 *Pd, float2 *P32, IpLds<MM> &w,
                                    double &ldet) {
    constexpr int M2 = M * M;
    constexpr int W = M + 1;  // row stride of the augmented matrix
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
            for (int k = 0; k < M; ++k) s = s + conjd(ld(Pd[k * M + r])) * ld(w.Qd[m * M2 + k * M + c]);
            w.A[r * W + c] = st(s);
            a2 = abs2(s);
        }
        if (lane < M) w.A[lane * W + M] = make_double2(lane == m ? 1.0 : 0.0, 0.0);
        const double amax2 = wave_max(a2);
        if (!(amax2 > 0.0) || !(amax2 < INFINITY)) return ST_SINGULAR;
#pragma unroll 1
        for (int k = 0; k < M; ++k) {
            int p = k;
            double best = abs2(ld(w.A[k * W + k]));
            for (int i = k + 1; i < M; ++i) {
                const double a = abs2(ld(w.A[i * W + k]));
                if (a > best) {
                    best = a;
                    p = i;
                }
            }
            if (!(best >= kPivotTol * kPivotTol * amax2)) return ST_SINGULAR;
            if (p != k && lane <= M) {
                const double2 t = w.A[k * W + lane];
                w.A[k * W + lane] = w.A[p * W + lane];
                w.A[p * W + lane] = t;
            }
            const cd piv = ld(w.A[k * W + k]);
            const cd ipiv = rcp_d(abs2(piv)) * conjd(piv);
            if (lane <= M) w.A[k * W + lane] = st(ld(w.A[k * W + lane]) * ipiv);
            if (lane < M) w.colk[lane] = w.A[lane * W + k];
            for (int i2 = lane; i2 < M * W; i2 += 64) {
                const int i = i2 / W, j = i2 % W;
                if (i != k) w.A[i * W + j] = st(ld(w.A[i * W + j]) - ld(w.colk[i]) * ld(w.A[k * W + j]));
            }
        }
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
    // ln|det P|^2: elimination with partial pivoting on a copy of P
    if (el) w.A[r * W + c] = Pd[lane];
    double acc = 0.0;
#pragma unroll 1
    for (int k = 0; k < M; ++k) {
        int p = k;
        double best = abs2(ld(w.A[k * W + k]));
        for (int i = k + 1; i < M; ++i) {
            const double a = abs2(ld(w.A[i * W + k]));
            if (a > best) {
                best = a;
                p = i;
            }
        }
        if (!(best > 0.0)) return ST_SINGULAR;
        acc += log(best);
        if (p != k && lane < M) {
            const double2 t = w.A[k * W + lane];
            w.A[k * W + lane] = w.A[p * W + lane];
            w.A[p * W + lane] = t;
        }
        const cd piv = ld(w.A[k * W + k]);
        const cd ipiv = rcp_d(abs2(piv)) * conjd(piv);
        if (lane < M) w.colk[lane] = st(ld(w.A[lane * W + k]) * ipiv);
        for (int i2 = lane; i2 < M * M; i2 += 64) {
            const int i = i2 / M, j = i2 % M;
            if (i > k) w.A[i * W + j] = st(ld(w.A[i * W + j]) - ld(w.colk[i]) * ld(w.A[k * W + j]));
        }
    }
    ldet = acc;
    if (el) {
        const double2 p = Pd[lane];
        P32[lane] = make_float2(static_cast<float>(p.x), static_cast<float>(p.y));
    }
    return ST_OK;
}

}  // namespace ffca
