/*
 * FastFCA reference oracle -- plain, slow, double precision, CPU only.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this library. The GPU library
 * shares no code, header, table or helper with this file.
 *
 * Source: Ito, Ikeshita, Sawada, Nakatani, "A Joint Diagonalization Based
 * Efficient Approach to Underdetermined Blind Audio Source Separation Using
 * the Multichannel Wiener Filter" (arXiv 2101.08563).
 *
 * Notation (paper -> here): frequency i -> f, frame j -> t, decorrelation
 * matrix W -> P (columns w_m = P[:,m]), [L]_{mn} = [Lambda_n]_{mm} -> lam[n][m],
 * [H]_{nj} = h_{jn} -> v[t][n], sigma^2_{mj} = [LH]_{mj} -> sigma2(m,t),
 * [U]_{mj} = |w_m^H x_j|^2 -> U[m][t].
 *
 * Every frequency is an independent problem (Sec. II; Sec. IV-G), so all
 * per-frequency routines take one frequency's arrays.
 *
 * Layouts (row-major, C order):
 *   x   [T][M]    complex   mixture STFT of one frequency
 *   P   [M][M]    complex   P[r][c]; column c is w_c
 *   lam [N][M]    real > 0
 *   v   [T][N]    real > 0
 *   U   [M][T]    real >= 0
 *   Q   [M][M][M] complex   Q[m][r][c] = [Q_m]_{rc}
 *
 * Floating point: IEEE double throughout; built without fast-math.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OFC_OK 0
#define OFC_E_ARG (-1)
#define OFC_E_NOMEM (-2)
#define OFC_E_SINGULAR (-4)

/* Relative pivot threshold below which a linear solve is declared singular. */
#define OFC_PIVOT_TOL 1e-12

/* sigma^2_{mt} = sum_n h_{tn} [Lambda_n]_{mm}  (Sec. IV-D, eq:sigmadef). */
static double sigma2_at(int M, int N, const double *lam, const double *vt, int m)
{
    double s = 0.0;
    for (int n = 0; n < N; ++n)
        s += vt[n] * lam[n * M + m];
    return s;
}

/*
 * Weighted covariances, all m at once (Sec. IV-E, eq:wsampcov; Algorithm 1,
 * first step of the loop over m). Q_m depends only on L and H, so computing
 * all of them before the IP sweep gives the same matrices.
 *   Q_m = (1/T) sum_t x_t x_t^H / sigma^2_{mt}
 */
void ofc_weighted_cov(int T, int M, int N, const cplx *x, const double *lam,
                      const double *v, cplx *Q)
{
    memset(Q, 0, sizeof(cplx) * (size_t)M * M * M);
    for (int t = 0; t < T; ++t) {
        const cplx *xt = x + (size_t)t * M;
        const double *vt = v + (size_t)t * N;
        for (int m = 0; m < M; ++m) {
            double w = 1.0 / sigma2_at(M, N, lam, vt, m);
            cplx *Qm = Q + (size_t)m * M * M;
            for (int r = 0; r < M; ++r)
                for (int c = 0; c < M; ++c)
                    Qm[r * M + c] += w * xt[r] * conj(xt[c]);
        }
    }
    for (int i = 0; i < M * M * M; ++i)
        Q[i] /= (double)T;
}

/*
 * Solve A z = b in place (A is n x n, row-major) by Gaussian elimination with
 * partial pivoting. A and b are overwritten; the solution is left in b.
 * Returns OFC_E_SINGULAR when a pivot is tiny relative to the largest entry.
 */
static int lu_solve(int n, cplx *A, cplx *b)
{
    double amax = 0.0;
    for (int i = 0; i < n * n; ++i)
        if (cabs(A[i]) > amax)
            amax = cabs(A[i]);
    if (!(amax > 0.0) || !isfinite(amax))
        return OFC_E_SINGULAR;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = cabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double a = cabs(A[i * n + k]);
            if (a > best) {
                best = a;
                p = i;
            }
        }
        if (best < OFC_PIVOT_TOL * amax)
            return OFC_E_SINGULAR;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                cplx tmp = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = tmp;
            }
            cplx tmp = b[k];
            b[k] = b[p];
            b[p] = tmp;
        }
        for (int i = k + 1; i < n; ++i) {
            cplx l = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j)
                A[i * n + j] -= l * A[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        cplx s = b[i];
        for (int j = i + 1; j < n; ++j)
            s -= A[i * n + j] * b[j];
        b[i] = s / A[i * n + i];
    }
    return OFC_OK;
}

/*
 * One IP column update (Sec. IV-E, eq:ip1 then eq:ip2):
 *   w_m <- (P^H Q_m)^{-1} e_m ;  w_m <- w_m / sqrt(w_m^H Q_m w_m)
 * P is updated in place (column m replaced).
 */
int ofc_ip_column(int M, cplx *P, const cplx *Qm, int m)
{
    if (M < 1 || M > 64 || m < 0 || m >= M)
        return OFC_E_ARG;
    cplx A[64 * 64];
    cplx w[64];
    /* A = P^H Q_m */
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < M; ++c) {
            cplx s = 0.0;
            for (int k = 0; k < M; ++k)
                s += conj(P[k * M + r]) * Qm[k * M + c];
            A[r * M + c] = s;
        }
    for (int r = 0; r < M; ++r)
        w[r] = (r == m) ? 1.0 : 0.0;
    int st = lu_solve(M, A, w);
    if (st != OFC_OK)
        return st;
    /* w^H Q_m w is real and positive for Hermitian PD Q_m. */
    cplx q = 0.0;
    for (int r = 0; r < M; ++r) {
        cplx s = 0.0;
        for (int c = 0; c < M; ++c)
            s += Qm[r * M + c] * w[c];
        q += conj(w[r]) * s;
    }
    double qr = creal(q);
    if (!(qr > 0.0) || !isfinite(qr))
        return OFC_E_SINGULAR;
    double inv = 1.0 / sqrt(qr);
    for (int r = 0; r < M; ++r)
        P[r * M + m] = w[r] * inv;
    return OFC_OK;
}

/* U_{mt} = |w_m^H x_t|^2  (Sec. IV-E, eq:Udef; Algorithm 1 update of U). */
void ofc_decorrelated_power(int T, int M, const cplx *P, const cplx *x, double *U)
{
    for (int t = 0; t < T; ++t) {
        const cplx *xt = x + (size_t)t * M;
        for (int m = 0; m < M; ++m) {
            cplx y = 0.0;
            for (int r = 0; r < M; ++r)
                y += conj(P[r * M + m]) * xt[r];
            U[(size_t)m * T + t] = creal(y) * creal(y) + cimag(y) * cimag(y);
        }
    }
}

/*
 * EM update of source n for the channel-time IS-NMF U ~ LH (Algorithm 1, the
 * body of the loop over n): posterior gain G_n and posterior power Phi_n from
 * the current L and H, then column n of L from Phi_n and the old row n of H,
 * then row n of H from Phi_n and the new column n of L.
 * phi is scratch of M*T doubles.
 */
void ofc_em_source(int T, int M, int N, const double *U, double *lam, double *v,
                   int n, double *phi)
{
    for (int t = 0; t < T; ++t) {
        const double *vt = v + (size_t)t * N;
        for (int m = 0; m < M; ++m) {
            double s2 = sigma2_at(M, N, lam, vt, m);
            double a = vt[n] * lam[n * M + m];
            double g = a / s2;
            phi[(size_t)m * T + t] = g * g * U[(size_t)m * T + t] + (1.0 - g) * a;
        }
    }
    for (int m = 0; m < M; ++m) {
        double s = 0.0;
        for (int t = 0; t < T; ++t)
            s += phi[(size_t)m * T + t] / v[(size_t)t * N + n];
        lam[n * M + m] = s / (double)T;
    }
    for (int t = 0; t < T; ++t) {
        double s = 0.0;
        for (int m = 0; m < M; ++m)
            s += phi[(size_t)m * T + t] / lam[n * M + m];
        v[(size_t)t * N + n] = s / (double)M;
    }
}

/*
 * MM update of L then H, all sources at once (Algorithm 2, the two
 * multiplicative square-root rules). scratch holds 2*M*T doubles.
 */
void ofc_mm_update(int T, int M, int N, const double *U, double *lam, double *v,
                   double *scratch)
{
    double *a = scratch;                 /* U / (LH)^2  [M][T] */
    double *b = scratch + (size_t)M * T; /* 1 / (LH)    [M][T] */
    for (int t = 0; t < T; ++t)
        for (int m = 0; m < M; ++m) {
            double s2 = sigma2_at(M, N, lam, v + (size_t)t * N, m);
            a[(size_t)m * T + t] = U[(size_t)m * T + t] / (s2 * s2);
            b[(size_t)m * T + t] = 1.0 / s2;
        }
    /* L <- L .* sqrt( (A H^T) ./ (B H^T) ) */
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < N; ++n) {
            double num = 0.0, den = 0.0;
            for (int t = 0; t < T; ++t) {
                num += a[(size_t)m * T + t] * v[(size_t)t * N + n];
                den += b[(size_t)m * T + t] * v[(size_t)t * N + n];
            }
            lam[n * M + m] *= sqrt(num / den);
        }
    /* H is updated from the new L. */
    for (int t = 0; t < T; ++t)
        for (int m = 0; m < M; ++m) {
            double s2 = sigma2_at(M, N, lam, v + (size_t)t * N, m);
            a[(size_t)m * T + t] = U[(size_t)m * T + t] / (s2 * s2);
            b[(size_t)m * T + t] = 1.0 / s2;
        }
    for (int t = 0; t < T; ++t)
        for (int n = 0; n < N; ++n) {
            double num = 0.0, den = 0.0;
            for (int m = 0; m < M; ++m) {
                num += lam[n * M + m] * a[(size_t)m * T + t];
                den += lam[n * M + m] * b[(size_t)m * T + t];
            }
            v[(size_t)t * N + n] *= sqrt(num / den);
        }
}

/* ln |det P|^2 by LU with partial pivoting. Returns -INFINITY if singular. */
double ofc_logabsdet2(int M, const cplx *P)
{
    cplx A[64 * 64];
    if (M < 1 || M > 64)
        return NAN;
    memcpy(A, P, sizeof(cplx) * (size_t)M * M);
    double acc = 0.0;
    for (int k = 0; k < M; ++k) {
        int p = k;
        double best = cabs(A[k * M + k]);
        for (int i = k + 1; i < M; ++i)
            if (cabs(A[i * M + k]) > best) {
                best = cabs(A[i * M + k]);
                p = i;
            }
        if (best == 0.0)
            return -INFINITY;
        if (p != k)
            for (int j = 0; j < M; ++j) {
                cplx tmp = A[k * M + j];
                A[k * M + j] = A[p * M + j];
                A[p * M + j] = tmp;
            }
        for (int i = k + 1; i < M; ++i) {
            cplx l = A[i * M + k] / A[k * M + k];
            for (int j = k; j < M; ++j)
                A[i * M + j] -= l * A[k * M + j];
        }
        acc += 2.0 * log(cabs(A[k * M + k]));
    }
    return acc;
}

/*
 * Per-frequency log-likelihood per TF bin, i.e. minus the negative
 * log-likelihood of Sec. IV-D (eq:negll) divided by T, with the constant
 * M ln(pi) per bin that eq:negll drops restored from the proper complex
 * Gaussian density of Sec. III-A:
 *   LL_f = ln|det P|^2 - (1/T) sum_{m,t} [ ln pi + ln sigma^2_{mt} + U_{mt}/sigma^2_{mt} ]
 */
double ofc_loglik_freq(int T, int M, int N, const cplx *x, const cplx *P,
                       const double *lam, const double *v)
{
    const double lnpi = log(3.14159265358979323846);
    double acc = 0.0;
    for (int t = 0; t < T; ++t) {
        const cplx *xt = x + (size_t)t * M;
        const double *vt = v + (size_t)t * N;
        for (int m = 0; m < M; ++m) {
            cplx y = 0.0;
            for (int r = 0; r < M; ++r)
                y += conj(P[r * M + m]) * xt[r];
            double u = creal(y) * creal(y) + cimag(y) * cimag(y);
            double s2 = sigma2_at(M, N, lam, vt, m);
            acc += lnpi + log(s2) + u / s2;
        }
    }
    return ofc_logabsdet2(M, P) - acc / (double)T;
}

/*
 * One iteration on one frequency. what: bit 0 = IP sweep over m = 1..M
 * (ascending, each solve seeing the columns already updated), bit 1 = update
 * of L and H. algo: 0 = EM (Algorithm 1, sources n = 1..N in order),
 * 1 = MM (Algorithm 2). U is always recomputed from the current P before the
 * L/H update. Qwork: M*M*M complex; dwork: 3*M*T doubles.
 */
int ofc_iterate_freq(int T, int M, int N, const cplx *x, cplx *P, double *lam,
                     double *v, int what, int algo, cplx *Qwork, double *dwork)
{
    if (what & 1) {
        ofc_weighted_cov(T, M, N, x, lam, v, Qwork);
        for (int m = 0; m < M; ++m) {
            int st = ofc_ip_column(M, P, Qwork + (size_t)m * M * M, m);
            if (st != OFC_OK)
                return st;
        }
    }
    if (what & 2) {
        double *U = dwork;
        double *scratch = dwork + (size_t)M * T;
        ofc_decorrelated_power(T, M, P, x, U);
        if (algo == 0) {
            for (int n = 0; n < N; ++n)
                ofc_em_source(T, M, N, U, lam, v, n, scratch);
        } else {
            ofc_mm_update(T, M, N, U, lam, v, scratch);
        }
    }
    return OFC_OK;
}

/*
 * Fit all F frequencies for n_iter iterations (IP then L/H update per
 * iteration). x [F][T][M], P [F][M][M], lam [F][N][M], v [F][T][N] updated in
 * place. ll_trace, if non-NULL, is [F][n_iter]: per-frequency LL after each
 * iteration. nthreads <= 0 means the OpenMP default. Returns the first error
 * status met (frequency order), OFC_OK otherwise.
 */
int ofc_fit(int F, int T, int M, int N, const cplx *x, cplx *P, double *lam,
            double *v, int n_iter, int algo, double *ll_trace, int nthreads)
{
    if (F < 1 || T < 1 || M < 1 || M > 64 || N < 1 || n_iter < 0)
        return OFC_E_ARG;
    int status = OFC_OK;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        cplx *Qw = (cplx *)malloc(sizeof(cplx) * (size_t)M * M * M);
        double *dw = (double *)malloc(sizeof(double) * 3 * (size_t)M * T);
#pragma omp for schedule(dynamic, 1)
        for (int f = 0; f < F; ++f) {
            if (!Qw || !dw) {
#pragma omp critical
                status = OFC_E_NOMEM;
                continue;
            }
            const cplx *xf = x + (size_t)f * T * M;
            cplx *Pf = P + (size_t)f * M * M;
            double *lf = lam + (size_t)f * N * M;
            double *vf = v + (size_t)f * T * N;
            for (int it = 0; it < n_iter; ++it) {
                int st = ofc_iterate_freq(T, M, N, xf, Pf, lf, vf, 3, algo, Qw, dw);
                if (st != OFC_OK) {
#pragma omp critical
                    if (status == OFC_OK)
                        status = st;
                    break;
                }
                if (ll_trace)
                    ll_trace[(size_t)f * n_iter + it] = ofc_loglik_freq(T, M, N, xf, Pf, lf, vf);
            }
        }
        free(Qw);
        free(dw);
    }
    return status;
}

/* Per-frequency LL for all F (see ofc_loglik_freq); returns the mean over f. */
double ofc_loglik(int F, int T, int M, int N, const cplx *x, const cplx *P,
                  const double *lam, const double *v, double *ll_f)
{
    double acc = 0.0;
    for (int f = 0; f < F; ++f) {
        double l = ofc_loglik_freq(T, M, N, x + (size_t)f * T * M, P + (size_t)f * M * M,
                                   lam + (size_t)f * N * M, v + (size_t)f * T * N);
        if (ll_f)
            ll_f[f] = l;
        acc += l;
    }
    return acc / (double)F;
}

/* Inverse of an M x M complex matrix by Gauss-Jordan with partial pivoting. */
static int invert(int M, const cplx *A_in, cplx *Ainv)
{
    cplx A[64 * 64];
    memcpy(A, A_in, sizeof(cplx) * (size_t)M * M);
    for (int i = 0; i < M * M; ++i)
        Ainv[i] = 0.0;
    for (int i = 0; i < M; ++i)
        Ainv[i * M + i] = 1.0;
    for (int k = 0; k < M; ++k) {
        int p = k;
        double best = cabs(A[k * M + k]);
        for (int i = k + 1; i < M; ++i)
            if (cabs(A[i * M + k]) > best) {
                best = cabs(A[i * M + k]);
                p = i;
            }
        if (best == 0.0)
            return OFC_E_SINGULAR;
        if (p != k)
            for (int j = 0; j < M; ++j) {
                cplx t1 = A[k * M + j];
                A[k * M + j] = A[p * M + j];
                A[p * M + j] = t1;
                cplx t2 = Ainv[k * M + j];
                Ainv[k * M + j] = Ainv[p * M + j];
                Ainv[p * M + j] = t2;
            }
        cplx d = A[k * M + k];
        for (int j = 0; j < M; ++j) {
            A[k * M + j] /= d;
            Ainv[k * M + j] /= d;
        }
        for (int i = 0; i < M; ++i) {
            if (i == k)
                continue;
            cplx l = A[i * M + k];
            for (int j = 0; j < M; ++j) {
                A[i * M + j] -= l * A[k * M + j];
                Ainv[i * M + j] -= l * Ainv[k * M + j];
            }
        }
    }
    return OFC_OK;
}

/*
 * Multichannel Wiener filter in the FastFCA form (Sec. IV-F, eq:Doclo):
 *   y_{n,t} = P^{-H} diag_m( h_{tn} lam_{nm} / sigma^2_{mt} ) P^H x_t
 * y is [N][F][T][M].
 */
int ofc_mwf(int F, int T, int M, int N, const cplx *x, const cplx *P,
            const double *lam, const double *v, cplx *y)
{
    if (M < 1 || M > 64)
        return OFC_E_ARG;
    for (int f = 0; f < F; ++f) {
        const cplx *Pf = P + (size_t)f * M * M;
        const double *lf = lam + (size_t)f * N * M;
        cplx Pinv[64 * 64];
        if (invert(M, Pf, Pinv) != OFC_OK)
            return OFC_E_SINGULAR;
        /* B = P^{-H}: B[r][c] = conj(Pinv[c][r]) */
        for (int t = 0; t < T; ++t) {
            const cplx *xt = x + ((size_t)f * T + t) * M;
            const double *vt = v + ((size_t)f * T + t) * N;
            cplx z[64];
            for (int m = 0; m < M; ++m) {
                cplx s = 0.0;
                for (int r = 0; r < M; ++r)
                    s += conj(Pf[r * M + m]) * xt[r];
                z[m] = s;
            }
            for (int n = 0; n < N; ++n) {
                cplx *yn = y + (((size_t)n * F + f) * T + t) * M;
                cplx gz[64];
                for (int m = 0; m < M; ++m) {
                    double s2 = sigma2_at(M, N, lf, vt, m);
                    gz[m] = (vt[n] * lf[n * M + m] / s2) * z[m];
                }
                for (int r = 0; r < M; ++r) {
                    cplx s = 0.0;
                    for (int c = 0; c < M; ++c)
                        s += conj(Pinv[c * M + r]) * gz[c];
                    yn[r] = s;
                }
            }
        }
    }
    return OFC_OK;
}

/* ------------------------------------------------------------------------
 * Piecewise stationary extension (Sec. VI, "Piecewise Stationary Extension
 * of FastFCA"). Frames are partitioned into J = T / B blocks of B consecutive
 * frames; within block j every frame has the covariance
 * sum_n h_{jn} P^{-H} Lambda_n P^{-1}. The cost eq:negllpws is minimized by
 * the same Algorithm 1 / Algorithm 2 with the input Xhat_j = (1/B) sum_b
 * x_j^(b) x_j^(b)H in place of x_j x_j^H, so that
 *   Q_m = (1/J) sum_j Xhat_j / sigma^2_{mj},  U_{mj} = w_m^H Xhat_j w_m
 * (the short-term power <|y_mj|^2>), and v is [J][N].
 * Layout: Xh [J][M][M] complex per frequency, [F][J][M][M] for all.
 * ------------------------------------------------------------------------ */

/* Xhat_j = (1/B) sum_{b<B} x_{jB+b} x_{jB+b}^H for one frequency; x [T][M], T = J B. */
void ofc_block_cov(int J, int B, int M, const cplx *x, cplx *Xh)
{
    for (int j = 0; j < J; ++j) {
        cplx *Xj = Xh + (size_t)j * M * M;
        for (int i = 0; i < M * M; ++i)
            Xj[i] = 0.0;
        for (int b = 0; b < B; ++b) {
            const cplx *xt = x + ((size_t)j * B + b) * M;
            for (int r = 0; r < M; ++r)
                for (int c = 0; c < M; ++c)
                    Xj[r * M + c] += xt[r] * conj(xt[c]);
        }
        for (int i = 0; i < M * M; ++i)
            Xj[i] /= (double)B;
    }
}

/* Q_m = (1/J) sum_j Xhat_j / sigma^2_{mj}, all m (eq:wsampcov with Xhat_j). */
void ofc_weighted_cov_blocks(int J, int M, int N, const cplx *Xh, const double *lam,
                             const double *v, cplx *Q)
{
    memset(Q, 0, sizeof(cplx) * (size_t)M * M * M);
    for (int j = 0; j < J; ++j) {
        const cplx *Xj = Xh + (size_t)j * M * M;
        const double *vj = v + (size_t)j * N;
        for (int m = 0; m < M; ++m) {
            double w = 1.0 / sigma2_at(M, N, lam, vj, m);
            cplx *Qm = Q + (size_t)m * M * M;
            for (int i = 0; i < M * M; ++i)
                Qm[i] += w * Xj[i];
        }
    }
    for (int i = 0; i < M * M * M; ++i)
        Q[i] /= (double)J;
}

/* U_{mj} = w_m^H Xhat_j w_m, the short-term power of y_m in block j. U [M][J]. */
void ofc_block_power(int J, int M, const cplx *P, const cplx *Xh, double *U)
{
    for (int j = 0; j < J; ++j) {
        const cplx *Xj = Xh + (size_t)j * M * M;
        for (int m = 0; m < M; ++m) {
            cplx q = 0.0;
            for (int r = 0; r < M; ++r) {
                cplx s = 0.0;
                for (int c = 0; c < M; ++c)
                    s += Xj[r * M + c] * P[c * M + m];
                q += conj(P[r * M + m]) * s;
            }
            U[(size_t)m * J + j] = creal(q);
        }
    }
}

/*
 * Per-frequency log-likelihood per frame of the piecewise stationary model:
 * minus eq:negllpws divided by J, with M ln(pi) restored,
 *   LL_f = ln|det P|^2 - (1/J) sum_{m,j} [ ln pi + ln sigma^2_{mj} + U_{mj}/sigma^2_{mj} ].
 */
double ofc_loglik_blocks_freq(int J, int M, int N, const cplx *Xh, const cplx *P,
                              const double *lam, const double *v)
{
    const double lnpi = log(3.14159265358979323846);
    double *U = (double *)malloc(sizeof(double) * (size_t)M * J);
    if (!U)
        return NAN;
    ofc_block_power(J, M, P, Xh, U);
    double acc = 0.0;
    for (int j = 0; j < J; ++j)
        for (int m = 0; m < M; ++m) {
            double s2 = sigma2_at(M, N, lam, v + (size_t)j * N, m);
            acc += lnpi + log(s2) + U[(size_t)m * J + j] / s2;
        }
    free(U);
    return ofc_logabsdet2(M, P) - acc / (double)J;
}

/* One iteration of the block model on one frequency (what, algo as in
 * ofc_iterate_freq). Qwork: M*M*M complex; dwork: 3*M*J doubles. */
int ofc_iterate_blocks_freq(int J, int M, int N, const cplx *Xh, cplx *P, double *lam,
                            double *v, int what, int algo, cplx *Qwork, double *dwork)
{
    if (what & 1) {
        ofc_weighted_cov_blocks(J, M, N, Xh, lam, v, Qwork);
        for (int m = 0; m < M; ++m) {
            int st = ofc_ip_column(M, P, Qwork + (size_t)m * M * M, m);
            if (st != OFC_OK)
                return st;
        }
    }
    if (what & 2) {
        double *U = dwork;
        double *scratch = dwork + (size_t)M * J;
        ofc_block_power(J, M, P, Xh, U);
        if (algo == 0) {
            for (int n = 0; n < N; ++n)
                ofc_em_source(J, M, N, U, lam, v, n, scratch);
        } else {
            ofc_mm_update(J, M, N, U, lam, v, scratch);
        }
    }
    return OFC_OK;
}

/*
 * Fit the block model on all F frequencies: x [F][T][M] with T = J B,
 * P [F][M][M], lam [F][N][M], v [F][J][N]; ll_trace [F][n_iter] or NULL.
 */
int ofc_fit_blocks(int F, int T, int M, int N, int B, const cplx *x, cplx *P, double *lam,
                   double *v, int n_iter, int algo, double *ll_trace, int nthreads)
{
    if (F < 1 || B < 1 || T < B || T % B != 0 || M < 1 || M > 64 || N < 1 || n_iter < 0)
        return OFC_E_ARG;
    const int J = T / B;
    int status = OFC_OK;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        cplx *Xh = (cplx *)malloc(sizeof(cplx) * (size_t)J * M * M);
        cplx *Qw = (cplx *)malloc(sizeof(cplx) * (size_t)M * M * M);
        double *dw = (double *)malloc(sizeof(double) * 3 * (size_t)M * J);
#pragma omp for schedule(dynamic, 1)
        for (int f = 0; f < F; ++f) {
            if (!Xh || !Qw || !dw) {
#pragma omp critical
                status = OFC_E_NOMEM;
                continue;
            }
            ofc_block_cov(J, B, M, x + (size_t)f * T * M, Xh);
            cplx *Pf = P + (size_t)f * M * M;
            double *lf = lam + (size_t)f * N * M;
            double *vf = v + (size_t)f * J * N;
            for (int it = 0; it < n_iter; ++it) {
                int st = ofc_iterate_blocks_freq(J, M, N, Xh, Pf, lf, vf, 3, algo, Qw, dw);
                if (st != OFC_OK) {
#pragma omp critical
                    if (status == OFC_OK)
                        status = st;
                    break;
                }
                if (ll_trace)
                    ll_trace[(size_t)f * n_iter + it] = ofc_loglik_blocks_freq(J, M, N, Xh, Pf, lf, vf);
            }
        }
        free(Xh);
        free(Qw);
        free(dw);
    }
    return status;
}

/* Mean over f of the block-model LL per frame (ll_f [F] optional). */
double ofc_loglik_blocks(int F, int T, int M, int N, int B, const cplx *x, const cplx *P,
                         const double *lam, const double *v, double *ll_f)
{
    if (B < 1 || T % B != 0)
        return NAN;
    const int J = T / B;
    cplx *Xh = (cplx *)malloc(sizeof(cplx) * (size_t)J * M * M);
    if (!Xh)
        return NAN;
    double acc = 0.0;
    for (int f = 0; f < F; ++f) {
        ofc_block_cov(J, B, M, x + (size_t)f * T * M, Xh);
        double l = ofc_loglik_blocks_freq(J, M, N, Xh, P + (size_t)f * M * M, lam + (size_t)f * N * M,
                                          v + (size_t)f * J * N);
        if (ll_f)
            ll_f[f] = l;
        acc += l;
    }
    free(Xh);
    return acc / (double)F;
}

/*
 * Multichannel Wiener filter of the block model (eq:Doclo applied to every
 * frame, with the block's h): y_{n,t} = P^{-H} diag_m(h_{jn} lam_{nm} /
 * sigma^2_{mj}) P^H x_t, j = t / B. v [F][J][N]; y [N][F][T][M].
 */
int ofc_mwf_blocks(int F, int T, int M, int N, int B, const cplx *x, const cplx *P,
                   const double *lam, const double *v, cplx *y)
{
    if (M < 1 || M > 64 || B < 1 || T % B != 0)
        return OFC_E_ARG;
    const int J = T / B;
    for (int f = 0; f < F; ++f) {
        const cplx *Pf = P + (size_t)f * M * M;
        const double *lf = lam + (size_t)f * N * M;
        cplx Pinv[64 * 64];
        if (invert(M, Pf, Pinv) != OFC_OK)
            return OFC_E_SINGULAR;
        for (int t = 0; t < T; ++t) {
            const cplx *xt = x + ((size_t)f * T + t) * M;
            const double *vj = v + ((size_t)f * J + t / B) * N;
            cplx z[64];
            for (int m = 0; m < M; ++m) {
                cplx s = 0.0;
                for (int r = 0; r < M; ++r)
                    s += conj(Pf[r * M + m]) * xt[r];
                z[m] = s;
            }
            for (int n = 0; n < N; ++n) {
                cplx *yn = y + (((size_t)n * F + f) * T + t) * M;
                cplx gz[64];
                for (int m = 0; m < M; ++m) {
                    double s2 = sigma2_at(M, N, lf, vj, m);
                    gz[m] = (vj[n] * lf[n * M + m] / s2) * z[m];
                }
                for (int r = 0; r < M; ++r) {
                    cplx s = 0.0;
                    for (int c = 0; c < M; ++c)
                        s += conj(Pinv[c * M + r]) * gz[c];
                    yn[r] = s;
                }
            }
        }
    }
    return OFC_OK;
}

/* ------------------------------------------------------------------------
 * FastMNMF (Sec. V, "FastMNMF: Full-band Extension of FastFCA"; appendix
 * "FastMNMF", eq:NMFconst2, eq:FastMNMFcost). The source powers are no
 * longer free: h_{ijn} = sum_k t_{ikn} v_{jkn}, with spectral patterns T_n
 * shared over frames and activations V_n shared over frequencies, so the
 * frequencies are coupled through V. The cost is eq:negll summed over
 * frequencies with that h. W_i is updated by IP (eq:ip1, eq:ip2) as in
 * FastFCA, and Lambda, T, V by majorization-minimization of the
 * Itakura-Saito part sum (U/sigma^2 + ln sigma^2): for a parameter theta
 * entering sigma^2_b = theta phi_b + (rest), the auxiliary function built from
 * the convexity of 1/sigma^2 and the concavity of ln sigma^2 is minimized by
 *   theta <- theta * sqrt( sum_b phi_b U_b / sigma_b^4 / sum_b phi_b / sigma_b^2 )
 * with sigma^2 from the current values. One iteration: IP for every i, U,
 * then Lambda, then T, then V, each from the latest values of the others.
 * Layouts (F frequencies i, T frames j): x [F][T][M], P [F][M][M],
 * lam [F][N][M], tp [F][K][N] (t_{ikn}), va [T][K][N] (v_{jkn}); h [F][T][N].
 * ------------------------------------------------------------------------ */

/* h_{ijn} = sum_k t_{ikn} v_{jkn} (eq:NMFconst2). */
void ofc_mnmf_h(int F, int T, int N, int K, const double *tp, const double *va, double *h)
{
    for (int i = 0; i < F; ++i)
        for (int j = 0; j < T; ++j)
            for (int n = 0; n < N; ++n) {
                double s = 0.0;
                for (int k = 0; k < K; ++k)
                    s += tp[((size_t)i * K + k) * N + n] * va[((size_t)j * K + k) * N + n];
                h[((size_t)i * T + j) * N + n] = s;
            }
}

/* LL per bin averaged over frequencies (eq:FastMNMFcost, sign flipped,
 * divided by F T, M ln pi restored); ll_f [F] optional. */
double ofc_mnmf_loglik(int F, int T, int M, int N, int K, const cplx *x, const cplx *P,
                       const double *lam, const double *tp, const double *va, double *ll_f)
{
    double *h = (double *)malloc(sizeof(double) * (size_t)F * T * N);
    if (!h)
        return NAN;
    ofc_mnmf_h(F, T, N, K, tp, va, h);
    double acc = 0.0;
    for (int i = 0; i < F; ++i) {
        double l = ofc_loglik_freq(T, M, N, x + (size_t)i * T * M, P + (size_t)i * M * M,
                                   lam + (size_t)i * N * M, h + (size_t)i * T * N);
        if (ll_f)
            ll_f[i] = l;
        acc += l;
    }
    free(h);
    return acc / (double)F;
}

/*
 * One FastMNMF iteration over all frequencies. what: bit 0 = IP sweep of
 * every W_i, bit 1 = Lambda, bit 2 = T, bit 3 = V (in that order).
 * Returns OFC_OK or the first IP failure.
 */
int ofc_mnmf_iterate(int F, int T, int M, int N, int K, const cplx *x, cplx *P, double *lam,
                     double *tp, double *va, int what)
{
    const size_t FT = (size_t)F * T;
    double *h = (double *)malloc(sizeof(double) * FT * N);
    double *U = (double *)malloc(sizeof(double) * FT * M);      /* [F][M][T] */
    double *s2 = (double *)malloc(sizeof(double) * FT * M);     /* [F][T][M] */
    cplx *Q = (cplx *)malloc(sizeof(cplx) * (size_t)M * M * M);
    double *num = (double *)malloc(sizeof(double) * (size_t)T * K * N);
    double *den = (double *)malloc(sizeof(double) * (size_t)T * K * N);
    int status = OFC_OK;
    if (!h || !U || !s2 || !Q || !num || !den) {
        status = OFC_E_NOMEM;
        goto done;
    }
#define SIG2()                                                                             \
    do {                                                                                   \
        ofc_mnmf_h(F, T, N, K, tp, va, h);                                                 \
        for (int i = 0; i < F; ++i)                                                        \
            for (int j = 0; j < T; ++j)                                                    \
                for (int m = 0; m < M; ++m)                                                \
                    s2[((size_t)i * T + j) * M + m] =                                      \
                        sigma2_at(M, N, lam + (size_t)i * N * M, h + ((size_t)i * T + j) * N, m); \
    } while (0)
    ofc_mnmf_h(F, T, N, K, tp, va, h);
    for (int i = 0; i < F; ++i) {
        const cplx *xi = x + (size_t)i * T * M;
        cplx *Pi = P + (size_t)i * M * M;
        if (what & 1) {
            ofc_weighted_cov(T, M, N, xi, lam + (size_t)i * N * M, h + (size_t)i * T * N, Q);
            for (int m = 0; m < M; ++m) {
                int st = ofc_ip_column(M, Pi, Q + (size_t)m * M * M, m);
                if (st != OFC_OK) {
                    status = st;
                    goto done;
                }
            }
        }
        ofc_decorrelated_power(T, M, Pi, xi, U + (size_t)i * M * T);
    }
    if (what & 2) { /* Lambda: phi = h_{ijn}, sums over j */
        SIG2();
        for (int i = 0; i < F; ++i)
            for (int n = 0; n < N; ++n)
                for (int m = 0; m < M; ++m) {
                    double a = 0.0, b = 0.0;
                    for (int j = 0; j < T; ++j) {
                        double s = s2[((size_t)i * T + j) * M + m];
                        double hh = h[((size_t)i * T + j) * N + n];
                        a += hh * U[((size_t)i * M + m) * T + j] / (s * s);
                        b += hh / s;
                    }
                    lam[((size_t)i * N + n) * M + m] *= sqrt(a / b);
                }
    }
    if (what & 4) { /* T: phi = lam_{imn} v_{jkn}, sums over j and m */
        SIG2();
        for (int i = 0; i < F; ++i)
            for (int k = 0; k < K; ++k)
                for (int n = 0; n < N; ++n) {
                    double a = 0.0, b = 0.0;
                    for (int j = 0; j < T; ++j)
                        for (int m = 0; m < M; ++m) {
                            double s = s2[((size_t)i * T + j) * M + m];
                            double phi = lam[((size_t)i * N + n) * M + m] * va[((size_t)j * K + k) * N + n];
                            a += phi * U[((size_t)i * M + m) * T + j] / (s * s);
                            b += phi / s;
                        }
                    tp[((size_t)i * K + k) * N + n] *= sqrt(a / b);
                }
    }
    if (what & 8) { /* V: phi = lam_{imn} t_{ikn}, sums over i and m */
        SIG2();
        for (size_t q = 0; q < (size_t)T * K * N; ++q)
            num[q] = den[q] = 0.0;
        for (int i = 0; i < F; ++i)
            for (int j = 0; j < T; ++j)
                for (int m = 0; m < M; ++m) {
                    double s = s2[((size_t)i * T + j) * M + m];
                    double u = U[((size_t)i * M + m) * T + j];
                    for (int k = 0; k < K; ++k)
                        for (int n = 0; n < N; ++n) {
                            double phi = lam[((size_t)i * N + n) * M + m] * tp[((size_t)i * K + k) * N + n];
                            num[((size_t)j * K + k) * N + n] += phi * u / (s * s);
                            den[((size_t)j * K + k) * N + n] += phi / s;
                        }
                }
        for (size_t q = 0; q < (size_t)T * K * N; ++q)
            va[q] *= sqrt(num[q] / den[q]);
    }
#undef SIG2
done:
    free(h);
    free(U);
    free(s2);
    free(Q);
    free(num);
    free(den);
    return status;
}

/* n_iter FastMNMF iterations; ll_trace [n_iter] (LL per bin after each) or NULL. */
int ofc_mnmf_fit(int F, int T, int M, int N, int K, const cplx *x, cplx *P, double *lam,
                 double *tp, double *va, int n_iter, double *ll_trace)
{
    if (F < 1 || T < 1 || M < 1 || M > 64 || N < 1 || K < 1 || n_iter < 0)
        return OFC_E_ARG;
    for (int it = 0; it < n_iter; ++it) {
        int st = ofc_mnmf_iterate(F, T, M, N, K, x, P, lam, tp, va, 15);
        if (st != OFC_OK)
            return st;
        if (ll_trace)
            ll_trace[it] = ofc_mnmf_loglik(F, T, M, N, K, x, P, lam, tp, va, NULL);
    }
    return OFC_OK;
}

int ofc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
