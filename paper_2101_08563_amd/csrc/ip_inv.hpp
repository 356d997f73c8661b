// IP sweep through inverses for the wide family (M <= 8), on one wavefront.
#pragma once

#include "device.hpp"
#include "internal.hpp"
#include "ip_common.hpp"

namespace ffca {

// Sum over the eight 8-lane groups of a wavefront: every lane ends with the
// sum over its position i = lane & 7 in the eight groups, the same bits in
// the eight lanes of a position. row_ror:8 adds the two groups of a 16-lane
// row, then v_permlane32_swap pairs lane i with lane i + 32 and
// v_permlane16_swap row 0 with row 1 and row 2 with row 3. Every lane must
// be active.
__device__ __forceinline__ double fold_groups8(double v) {
    v += dpp_d<0x128>(v);
    unsigned lo = static_cast<unsigned>(static_cast<unsigned long long>(__double_as_longlong(v)));
    unsigned hi = static_cast<unsigned>(static_cast<unsigned long long>(__double_as_longlong(v)) >> 32);
    const auto l32 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h32 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    v = join_d(l32[0], h32[0]) + join_d(l32[1], h32[1]);
    lo = static_cast<unsigned>(static_cast<unsigned long long>(__double_as_longlong(v)));
    hi = static_cast<unsigned>(static_cast<unsigned long long>(__double_as_longlong(v)) >> 32);
    const auto l16 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h16 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return join_d(l16[0], h16[0]) + join_d(l16[1], h16[1]);
}
__device__ __forceinline__ cd fold_groups8(cd v) { return cmk(fold_groups8(v.re), fold_groups8(v.im)); }

// Doubles of LDS scratch ip_inv<M> needs: two copies of the matrices, the
// normalized pivot rows and pivot reciprocals of a step, the largest diagonal
// entry of each Q_m, and the column difference a.
template <int M>
constexpr int ip_inv_scratch_doubles() {
    return 2 * 2 * (M * M * M + 2 * M * M) + 2 * (M * M + 2 * M) + 2 * (M + 1) + M + (M & 1) + 2 * M;
}

// The IP sweep (eq:ip1, eq:ip2) for m = 1..M in order, by the algebra of
// ip_sm.hpp: w_m = u / sqrt(b^H u) with u = Q_m^{-1} b and b = P^{-H} e_m; the
// inverses of the Q_m and of P come from one Gauss-Jordan run on all of them
// at once (without pivoting for the Hermitian Q_m, whose pivots are Schur
// complements; with partial pivoting on [P | I]); replacing column m of P by
// w_m updates P^{-1} by Sherman-Morrison and det P by the matrix determinant
// lemma. For up to eight channels a matrix has up to 64 entries, so every lane
// holds several entries per elimination step. A step first writes the pivot
// rows divided by their pivots (M + 1 rows: one per Q_m, and P's after the
// row swap) and the pivot reciprocals, one or two entries per lane, so that
// the update of an entry is one complex multiply-add; and instead of keeping
// the new values in registers until all reads of the step are done, it reads
// one LDS copy of the matrices and writes the other (`scratch`, in LDS,
// caller-provided and 16-byte aligned, ip_inv_scratch_doubles<M>() doubles;
// the wavefront's LDS instructions execute in order, so no barrier is
// needed). The sums of
// the sweep run with lane (group c = lane >> 3, position r = lane & 7) on the
// pair (r, c) and fold over the eight groups. qtot: the Q_m as Hermitian real
// parameters (M diagonal entries, then re/im of the upper triangle), already
// divided by T. Singular and non-finite cases are reported as in ip_sm.
// P (Pd) is updated in place and copied to P32; ldet = ln|det P|^2.
template <int M>
__device__ __noinline__ int ip_inv(const double *qtot, double2 *Pd, float2 *P32, double *scratch, double &ldet) {
    static_assert(M >= 2 && M <= 8, "ip_inv shape");
    constexpr int M2 = M * M;
    constexpr int W2 = 2 * M;
    constexpr int NQ = M * M2;          // entries of the Q_m
    constexpr int NE = NQ + M * W2;     // and of [P | I]
    constexpr int NS = (NE + 63) / 64;  // entries per lane
    const int lane = threadIdx.x & 63;
    constexpr int NR = M * M + W2;      // entries of the M + 1 pivot rows
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) d2 lds_d2;
    double2 *buf0 = reinterpret_cast<double2 *>(scratch);
    double2 *buf1 = buf0 + NE;
    double2 *prow_n = buf1 + NE;        // pivot rows over their pivots: Q_t's at t M, P's at M^2
    double2 *ipiv_n = prow_n + NR;      // 1 / pivot of Q_t at t, of P at M
    double *esc = reinterpret_cast<double *>(ipiv_n + M + 1);  // largest diagonal entry of each Q_m
    double2 *av = reinterpret_cast<double2 *>(esc + M + (M & 1));  // w_m - p_m (16-byte aligned)

    // entry e < NQ: Q_t (i, j) at e = t M^2 + i M + j; else [P | I] (i, j) at
    // NQ + i 2M + j
    double pmax = 0.0;
    bool finite = true;
    if (lane < M) {
        const double *qm = qtot + lane * M2;
        double d = 0.0;
#pragma unroll
        for (int r = 0; r < M; ++r) d = fmax(d, qm[r]);
        esc[lane] = d;
        finite = finite && d < INFINITY;
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int e = lane + 64 * q;
        if (e >= NE) continue;
        double2 v;
        if (e < NQ) {
            const int t = e / M2, i = (e / M) % M, j = e % M;
            const double *qm = qtot + t * M2;
            if (i == j) {
                v = make_double2(qm[i], 0.0);
            } else {
                const int lo = i < j ? i : j, hi = i < j ? j : i;
                const int p = upper_index<M>(lo, hi);
                v = make_double2(qm[M + 2 * p], i < j ? qm[M + 2 * p + 1] : -qm[M + 2 * p + 1]);
            }
            finite = finite && fabs(v.x) < INFINITY && fabs(v.y) < INFINITY;
        } else {
            const int i = (e - NQ) / W2, j = (e - NQ) % W2;
            v = j < M ? Pd[i * M + j] : make_double2(j - M == i ? 1.0 : 0.0, 0.0);
            pmax = fmax(pmax, abs2(ld(v)));
        }
        buf0[e] = v;
    }
    const double pscale = wave_max(pmax);
    finite = finite && pscale < INFINITY;
    if (__any(!finite)) return ST_NONFINITE;
    if (!(pscale > 0.0)) return ST_SINGULAR;

    // ---- the eliminations, step k on every matrix at once, src -> dst
    double mant = 1.0;  // |det P|^2 as mantissa and binary exponent
    int ex = 0;
    bool sing = false;
    const double2 *src = buf0;
    double2 *dst = buf1;
    // LDS views of the buffers (32-bit addresses, no generic-pointer checks)
    const lds_d2 *Rn = (const lds_d2 *)prow_n;  // the pivot rows, then the reciprocals at NR
    const lds_d2 *src_l = (const lds_d2 *)buf0;
    lds_d2 *dst_l = (lds_d2 *)buf1;
#pragma unroll 1
    for (int k = 0; k < M && !sing; ++k) {
        const double2 *X = src + NQ;
        // P's pivot row: the largest modulus in column k at or below row k
        int p = k;
        double best = abs2(ld(X[k * W2 + k]));
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const double a = abs2(ld(X[i * W2 + k]));
            if (i > k && a > best) {
                best = a;
                p = i;
            }
        }
        int e2;
        mant = frexp(mant * best, &e2);
        ex += e2;
        // the pivot rows over their pivots, and the reciprocals
        bool qbad = false;
#pragma unroll
        for (int q = 0; q < (NR + 63) / 64; ++q) {
            const int f = lane + 64 * q;
            if (f >= NR) continue;
            const bool fq = f < M * M;
            const int t = fq ? f / M : M, j = fq ? f % M : f - M * M;
            const cd piv = fq ? ld(src[t * M2 + k * M + k]) : ld(X[p * W2 + k]);
            const cd prw = fq ? ld(src[t * M2 + k * M + j]) : ld(X[p * W2 + j]);
            const cd ip = rcp_d(abs2(piv)) * conjd(piv);
            prow_n[f] = st(prw * ip);
            if (j == 0) ipiv_n[t] = st(ip);
            if (fq && j == 0) qbad = !(piv.re >= kPivotTol * esc[t]);
        }
        // every entry: one multiply-add with the normalized pivot row,
        //   new = (row k) ? r : base - c r,
        // with c the entry's column-k element, r the normalized pivot row's
        // element (for column k of a Q_m, which takes column k of the
        // inverse in place: the pivot reciprocal) and base the entry itself
        // (zero for column k of a Q_m). The entries go in batches of four whose
        // LDS reads are all issued before any is used; no lane branches.
        {
            const lds_d2 *S = src_l;
            lds_d2 *D = dst_l;
            constexpr int B = 4;
#pragma unroll
            for (int q0 = 0; q0 < NS; q0 += B) {
                d2 av[B], cv[B], rv[B];
                bool rowk[B], zero[B], live[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    if (q0 + u >= NS) break;
                    const int e0 = lane + 64 * (q0 + u);
                    live[u] = e0 < NE;
                    const int e = live[u] ? e0 : 0;
                    const bool isq = e < NQ;
                    const int fq = isq ? e : e - NQ;
                    const int t = fq / M2, i = isq ? (fq / M) % M : fq / W2, j = isq ? fq % M : fq % W2;
                    const int s_ = i == k ? p : (i == p ? k : i);  // P's rows, swapped
                    const int rowbase = isq ? t * M2 + i * M : NQ + s_ * W2;
                    rowk[u] = i == k;
                    zero[u] = isq && j == k;
                    const int ri = isq ? (j == k ? NR + t : t * M + j) : M * M + j;
                    av[u] = S[rowbase + j];
                    cv[u] = S[rowbase + k];
                    rv[u] = Rn[ri];
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    if (q0 + u >= NS) break;
                    const cd r = cmk(rv[u].x, rv[u].y);
                    const cd base = zero[u] ? cmk(0.0, 0.0) : cmk(av[u].x, av[u].y);
                    const cd nv = rowk[u] ? r : base - cmk(cv[u].x, cv[u].y) * r;
                    if (live[u]) D[lane + 64 * (q0 + u)] = d2{nv.re, nv.im};
                }
            }
        }
        sing = __any(qbad) || !(best >= kPivotTol * kPivotTol * pscale);
        const double2 *t = src;
        src = dst;
        dst = const_cast<double2 *>(t);
        const lds_d2 *tl = src_l;
        src_l = dst_l;
        dst_l = const_cast<lds_d2 *>(tl);
    }
    if (sing) return ST_SINGULAR;

    // ---- the sweep; src holds the Q_m^{-1} and, in the right half of X,
    // G = P^{-1}. Lane (group c, position r) handles the pair (r, c); the sums
    // over c of u = Q_m^{-1} b and of G a fold over the eight groups, leaving
    // entry r in position r of every group.
    const double2 *Qi = src;
    double2 *X = const_cast<double2 *>(src) + NQ;
    const int r = lane & 7, c = lane >> 3;
    const bool rc = r < M && c < M;
    const int rr = r < M ? r : 0, cc = c < M ? c : 0;
#pragma unroll 1
    for (int m = 0; m < M; ++m) {
        const cd qv = ld(Qi[m * M2 + rr * M + cc]);
        const cd gmc = ld(X[m * W2 + M + cc]);
        const cd gmr = ld(X[m * W2 + M + rr]);
        const cd grc = ld(X[rr * W2 + M + cc]);
        const cd pold = ld(Pd[rr * M + m]);
        // u_r = sum_c Q_m^{-1}[r][c] b_c with b = P^{-H} e_m = conj(row m of G)
        const cd u = fold_groups8(rc ? qv * conjd(gmc) : cmk(0.0, 0.0));
        // b^H u over the M positions of group 0 (the other lanes add zero),
        // made uniform across the wavefront
        const double s = readlane_d(row_sum(r < M && c == 0 ? (gmr * u).re : 0.0), 0);
        if (!(s > 0.0) || !(s < INFINITY)) return ST_SINGULAR;
        const cd wr = rsqrt_d(s) * u;
        if (r < M && c == 0) {
            Pd[r * M + m] = st(wr);
            av[r] = st(wr - pold);
        }
        // (G a)_r, a = w_m - p_m
        const cd ga = fold_groups8(rc ? grc * ld(av[cc]) : cmk(0.0, 0.0));
        // G <- G - (G a)(row m of G) / (1 + (G a)_m), det P *= 1 + (G a)_m
        const cd den = cmk(1.0 + readlane_d(ga.re, m), readlane_d(ga.im, m));
        const double den2 = abs2(den);
        if (!(den2 > 0.0) || !(den2 < INFINITY)) return ST_SINGULAR;
        int e2;
        mant = frexp(mant * den2, &e2);
        ex += e2;
        const cd idn = rcp_d(den2) * conjd(den);
        if (rc) X[r * W2 + M + c] = st(grc - ga * (gmc * idn));
    }
    ldet = log(mant) + static_cast<double>(ex) * 0.69314718055994531;
    if (lane < M2) {
        const double2 pv = Pd[lane];
        P32[lane] = make_float2(static_cast<float>(pv.x), static_cast<float>(pv.y));
    }
    return ST_OK;
}

}  // namespace ffca
