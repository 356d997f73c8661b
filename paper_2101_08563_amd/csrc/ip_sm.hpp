// IP sweep for M = 3, 4 through inverses, on one wavefront.
#pragma once

#include "device.hpp"
#include "internal.hpp"
#include "ip_common.hpp"

namespace ffca {

// Sum over the four 16-lane rows: every lane ends with v[i] + v[i + 16] +
// v[i + 32] + v[i + 48] for its position i in the row, the same bits in the
// four lanes of a position. v_permlane32_swap pairs lane i with lane i + 32,
// then v_permlane16_swap row 0 with row 1 and row 2 with row 3. Every lane
// must be active.
__device__ __forceinline__ double fold_rows(double v) {
    auto halves = [](double x, unsigned &lo, unsigned &hi) {
        const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
        lo = static_cast<unsigned>(b);
        hi = static_cast<unsigned>(b >> 32);
    };
    auto join = [](unsigned lo, unsigned hi) {
        return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
    };
    unsigned lo, hi;
    halves(v, lo, hi);
    const auto l32 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h32 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    v = join(l32[0], h32[0]) + join(l32[1], h32[1]);
    halves(v, lo, hi);
    const auto l16 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h16 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return join(l16[0], h16[0]) + join(l16[1], h16[1]);
}
__device__ __forceinline__ cd fold_rows(cd v) { return cmk(fold_rows(v.re), fold_rows(v.im)); }

// LDS work space of ip_sm for M <= MM.
template <int MM>
struct IpSmLds {
    double2 Q[MM][MM][MM];  // the Q_m, inverted in place
    double2 X[MM][2 * MM];  // [P | I], reduced to [I | P^{-1}]
    double2 av[MM];         // w_m minus the old column m of P
};

// The IP sweep (eq:ip1, eq:ip2) for m = 1..M in order. The solution of
// (P^H Q_m) w = e_m is w = Q_m^{-1} b with b = P^{-H} e_m, and eq:ip2's
// normalization w^H Q_m w = b^H Q_m^{-1} b makes
//   w_m = u / sqrt(b^H u),  u = Q_m^{-1} b.
// The Q_m do not change during the sweep, so their inverses and P^{-1} come
// from one elimination run on all of them at once, one entry per lane and
// slot: Gauss-Jordan in place without pivoting for the Hermitian positive
// semidefinite Q_m (their pivots are Schur complements, positive unless Q_m is
// singular), and Gauss-Jordan with partial pivoting on [P | I]. A step is one
// LDS round trip for P's pivot column and one for the entries each lane's new
// value needs (the row swap folded in). Replacing column m of P by w_m is the
// rank-one change P + a e_m^T, a = w_m - p_m, so
//   P^{-1} <- P^{-1} - (P^{-1} a)(e_m^T P^{-1}) / (1 + e_m^T P^{-1} a)
// (Sherman-Morrison), and det P is multiplied by the same denominator (matrix
// determinant lemma): two LDS round trips per column. ln|det P|^2 is one
// logarithm of the product of the squared pivot and denominator moduli.
// qtot: the M weighted covariances Q_m as Hermitian real parameters (M
// diagonal entries, then re/im of the upper triangle), already divided by T.
// A pivot of Q_m below tol times its largest diagonal entry, a pivot of P
// below tol times its largest entry, a non-positive b^H u or a zero
// denominator is reported as singular; a non-finite Q_m or P as non-finite.
// P (Pd) is updated in place and copied to P32.
template <int M, int MM>
__device__ __noinline__ int ip_sm(const double *qtot, double2 *Pd, float2 *P32, IpSmLds<MM> &w, double &ldet) {
    static_assert(M >= 2 && M <= MM, "ip_sm shape");
    static_assert(M <= 4, "the sums over c fold over the four 16-lane rows");
    constexpr int M2 = M * M;
    constexpr int W2 = 2 * M;
    constexpr int NQ = M * M2;           // entries of the Q_m
    constexpr int NE = NQ + M * W2;      // and of [P | I]
    constexpr int NS = (NE + 63) / 64;   // entries per lane
    const int lane = threadIdx.x & 63;

    // entry e < NQ: Q_t (i, j); else [P | I] (i, j). Lanes past NE take
    // entry 0 of Q_0 for their reads and store nothing.
    int et[NS], ei[NS], ej[NS];
    bool eq[NS], ein[NS];
    double esc[NS];  // for Q entries: the largest diagonal entry of Q_t
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int e = lane + 64 * q;
        ein[q] = e < NE;
        eq[q] = e < NQ || !ein[q];
        const int ee = ein[q] ? e : 0;
        if (eq[q]) {
            et[q] = ee / M2;
            ei[q] = (ee / M) % M;
            ej[q] = ee % M;
        } else {
            et[q] = M;
            ei[q] = (ee - NQ) / W2;
            ej[q] = (ee - NQ) % W2;
        }
    }
    double pmax = 0.0;  // largest squared modulus of this lane's entries of P
    bool finite = true;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int t = et[q], i = ei[q], j = ej[q];
        double2 v;
        if (eq[q]) {
            const double *qm = qtot + t * M2;
            double d = 0.0;
#pragma unroll
            for (int r = 0; r < M; ++r) d = fmax(d, qm[r]);
            esc[q] = d;
            if (i == j) {
                v = make_double2(qm[i], 0.0);
            } else {
                const int lo = i < j ? i : j, hi = i < j ? j : i;
                const int p = upper_index<M>(lo, hi);
                v = make_double2(qm[M + 2 * p], i < j ? qm[M + 2 * p + 1] : -qm[M + 2 * p + 1]);
            }
            finite = finite && fabs(v.x) < INFINITY && fabs(v.y) < INFINITY && d < INFINITY;
            if (ein[q]) w.Q[t][i][j] = v;
        } else {
            esc[q] = 0.0;
            v = j < M ? Pd[i * M + j] : make_double2(j - M == i ? 1.0 : 0.0, 0.0);
            pmax = fmax(pmax, abs2(ld(v)));
            w.X[i][j] = v;
        }
    }
    const double pscale = wave_max(pmax);
    finite = finite && pscale < INFINITY;
    if (__any(!finite)) return ST_NONFINITE;
    if (!(pscale > 0.0)) return ST_SINGULAR;

    // ---- the eliminations, step k on every matrix at once
    double mant = 1.0;  // |det P|^2 as mantissa and binary exponent
    int ex = 0;
    bool sing = false;
    auto step = [&](int k) {
        // P's pivot row: the largest modulus in column k at or below row k
        double colv[M];
#pragma unroll
        for (int i = 0; i < M; ++i) colv[i] = abs2(ld(w.X[i][k]));
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
        int e2;
        mant = frexp(mant * best, &e2);
        ex += e2;
        bool qbad = false;
        cd nv[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int t = et[q], i = ei[q], j = ej[q];
            cd arow, acol, prow, piv;
            if (eq[q]) {
                arow = ld(w.Q[t][i][j]);
                acol = ld(w.Q[t][i][k]);
                prow = ld(w.Q[t][k][j]);
                piv = ld(w.Q[t][k][k]);
            } else {
                const int src = i == k ? p : (i == p ? k : i);
                arow = ld(w.X[src][j]);
                acol = ld(w.X[src][k]);
                prow = ld(w.X[p][j]);
                piv = ld(w.X[p][k]);
            }
            const cd ipiv = rcp_d(abs2(piv)) * conjd(piv);
            const cd pr = prow * ipiv;
            nv[q] = i == k ? pr : arow - acol * pr;
            if (eq[q]) {
                // in place: column k of the inverse replaces column k
                if (j == k) nv[q] = i == k ? ipiv : cmk(0.0, 0.0) - acol * ipiv;
                qbad = qbad || (ein[q] && !(piv.re >= kPivotTol * esc[q]));
            }
        }
        sing = sing || __any(qbad) || !(best >= kPivotTol * kPivotTol * pscale);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            if (!ein[q]) continue;
            if (eq[q])
                w.Q[et[q]][ei[q]][ej[q]] = st(nv[q]);
            else
                w.X[ei[q]][ej[q]] = st(nv[q]);
        }
    };
    // the loop over k is unrolled except for M = 3, whose kernels would lose
    // their third wave per SIMD to the registers
    if constexpr (M == 3) {
#pragma unroll 1
        for (int k = 0; k < M && !sing; ++k) step(k);
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k)
            if (!sing) step(k);
    }
    if (sing) return ST_SINGULAR;

    // ---- the sweep; Q holds the Q_m^{-1}, the right half of X G = P^{-1}.
    // Lane (row c, position r) of the wavefront handles the pair (r, c): the
    // sums over c of u = Q_m^{-1} b and of G a are folded across the four
    // 16-lane rows, leaving entry r in position r of every row.
    const int r = lane & 15, c = lane >> 4;
    const bool rc = r < M && c < M;
    const int rr = r < M ? r : 0, cc = c < M ? c : 0;
#pragma unroll 1
    for (int m = 0; m < M; ++m) {
        const cd qv = ld(w.Q[m][rr][cc]);
        const cd gmc = ld(w.X[m][M + cc]);
        const cd gmr = ld(w.X[m][M + rr]);
        const cd grc = ld(w.X[rr][M + cc]);
        const cd pold = ld(Pd[rr * M + m]);
        // u_r = sum_c Q_m^{-1}[r][c] b_c with b = P^{-H} e_m = conj(row m of G)
        const cd u = fold_rows(rc ? qv * conjd(gmc) : cmk(0.0, 0.0));
        // b^H u over the M positions of row 0 (the other lanes add zero),
        // made uniform across the wavefront
        const double s = readlane_d(row_sum(r < M && c == 0 ? (gmr * u).re : 0.0), 0);
        if (!(s > 0.0) || !(s < INFINITY)) return ST_SINGULAR;
        const cd wr = rsqrt_d(s) * u;
        if (r < M && c == 0) {
            Pd[r * M + m] = st(wr);
            w.av[r] = st(wr - pold);
        }
        // (G a)_r, a = w_m - p_m
        const cd ga = fold_rows(rc ? grc * ld(w.av[cc]) : cmk(0.0, 0.0));
        // G <- G - (G a)(row m of G) / (1 + (G a)_m), det P *= 1 + (G a)_m
        const cd den = cmk(1.0 + readlane_d(ga.re, m), readlane_d(ga.im, m));
        const double den2 = abs2(den);
        if (!(den2 > 0.0) || !(den2 < INFINITY)) return ST_SINGULAR;
        int e2;
        mant = frexp(mant * den2, &e2);
        ex += e2;
        const cd idn = rcp_d(den2) * conjd(den);
        if (rc) w.X[r][M + c] = st(grc - ga * (gmc * idn));
    }
    ldet = log(mant) + static_cast<double>(ex) * 0.69314718055994531;
    if (lane < M2) {
        const double2 pv = Pd[lane];
        P32[lane] = make_float2(static_cast<float>(pv.x), static_cast<float>(pv.y));
    }
    return ST_OK;
}

}  // namespace ffca
