/*
 * Drives every entry point of the FP64 oracle (oracle/fastfca_oracle.c) on
 * small seeded inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py). Test
 * infrastructure: checks memory safety and undefined behaviour of the
 * oracle's code paths, not its numbers (those are pinned elsewhere).
 * Exit status 0 when every call returned and no sanitizer fired.
 */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void ofc_weighted_cov(int T, int M, int N, const cplx *x, const double *lam, const double *v, cplx *Q);
int ofc_ip_column(int M, cplx *P, const cplx *Qm, int m);
void ofc_decorrelated_power(int T, int M, const cplx *P, const cplx *x, double *U);
void ofc_em_source(int T, int M, int N, const double *U, double *lam, double *v, int n, double *sig2);
void ofc_mm_update(int T, int M, int N, const double *U, double *lam, double *v, double *work);
double ofc_logabsdet2(int M, const cplx *P);
double ofc_loglik_freq(int T, int M, int N, const cplx *x, const cplx *P, const double *lam, const double *v);
int ofc_fit(int F, int T, int M, int N, const cplx *x, cplx *P, double *lam, double *v, int n_iter, int algo,
            double *ll_trace, int nthreads);
double ofc_loglik(int F, int T, int M, int N, const cplx *x, const cplx *P, const double *lam, const double *v,
                  double *ll_f);
int ofc_mwf(int F, int T, int M, int N, const cplx *x, const cplx *P, const double *lam, const double *v, cplx *y);
int ofc_fit_blocks(int F, int T, int M, int N, int B, const cplx *x, cplx *P, double *lam, double *v, int n_iter,
                   int algo, double *ll_trace, int nthreads);
double ofc_loglik_blocks(int F, int T, int M, int N, int B, const cplx *x, const cplx *P, const double *lam,
                         const double *v, double *ll_f);
int ofc_mwf_blocks(int F, int T, int M, int N, int B, const cplx *x, const cplx *P, const double *lam,
                   const double *v, cplx *y);
double ofc_mnmf_loglik(int F, int T, int M, int N, int K, const cplx *x, const cplx *P, const double *lam,
                       const double *tp, const double *va, double *ll_f);
int ofc_mnmf_fit(int F, int T, int M, int N, int K, const cplx *x, cplx *P, double *lam, double *tp, double *va,
                 int n_iter, double *ll_trace);

static uint64_t state = 0x9E3779B97F4A7C15ULL;
static double uniform(void)  /* xorshift64*, in (0, 1) */
{
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return ((double)((state * 0x2545F4914F6CDD1DULL) >> 11) + 0.5) / 9007199254740992.0;
}

static void *must(size_t n)
{
    void *p = calloc(n, 1);
    if (!p) {
        fprintf(stderr, "allocation of %zu bytes failed\n", n);
        exit(2);
    }
    return p;
}

static int run(int F, int T, int M, int N, int B, int K)
{
    const int J = T / B;
    cplx *x = must(sizeof(cplx) * F * T * M);
    cplx *P = must(sizeof(cplx) * F * M * M);
    double *lam = must(sizeof(double) * F * N * M);
    double *v = must(sizeof(double) * F * T * N);
    double *vb = must(sizeof(double) * F * J * N);
    cplx *y = must(sizeof(cplx) * N * F * T * M);
    double *tr = must(sizeof(double) * F * 4);
    double *llf = must(sizeof(double) * F);
    cplx *Q = must(sizeof(cplx) * M * M * M);
    double *U = must(sizeof(double) * T * M);
    double *work = must(sizeof(double) * (4 * T * M + 4 * N * M + 16));
    double *sig2 = must(sizeof(double) * T * M);
    double *tp = must(sizeof(double) * F * K * N);
    double *va = must(sizeof(double) * T * K * N);
    for (int i = 0; i < F * T * M; ++i) x[i] = (uniform() - 0.5) + I * (uniform() - 0.5);
    for (int i = 0; i < F * N * M; ++i) lam[i] = 0.5 + uniform();
    for (int i = 0; i < F * T * N; ++i) v[i] = 0.5 + uniform();
    for (int i = 0; i < F * J * N; ++i) vb[i] = 0.5 + uniform();
    for (int i = 0; i < F * K * N; ++i) tp[i] = 0.5 + uniform();
    for (int i = 0; i < T * K * N; ++i) va[i] = 0.5 + uniform();
    for (int f = 0; f < F; ++f)
        for (int r = 0; r < M; ++r) P[(f * M + r) * M + r] = 1.0;
    int bad = 0;
    /* per-frequency pieces on frequency 0 */
    ofc_weighted_cov(T, M, N, x, lam, v, Q);
    for (int m = 0; m < M; ++m) bad |= ofc_ip_column(M, P, Q, m) != 0;
    ofc_decorrelated_power(T, M, P, x, U);
    for (int n = 0; n < N; ++n) ofc_em_source(T, M, N, U, lam, v, n, sig2);
    ofc_mm_update(T, M, N, U, lam, v, work);
    (void)ofc_logabsdet2(M, P);
    (void)ofc_loglik_freq(T, M, N, x, P, lam, v);
    /* whole fits: Algorithms 1 and 2, the block model, FastMNMF */
    bad |= ofc_fit(F, T, M, N, x, P, lam, v, 4, 0, tr, 1) != 0;
    bad |= ofc_fit(F, T, M, N, x, P, lam, v, 2, 1, NULL, 2) != 0;
    (void)ofc_loglik(F, T, M, N, x, P, lam, v, llf);
    bad |= ofc_mwf(F, T, M, N, x, P, lam, v, y) != 0;
    for (int f = 0; f < F; ++f)
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) P[(f * M + r) * M + c] = (r == c) ? 1.0 : 0.0;
    bad |= ofc_fit_blocks(F, T, M, N, B, x, P, lam, vb, 3, 0, tr, 1) != 0;
    (void)ofc_loglik_blocks(F, T, M, N, B, x, P, lam, vb, llf);
    bad |= ofc_mwf_blocks(F, T, M, N, B, x, P, lam, vb, y) != 0;
    for (int f = 0; f < F; ++f)
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) P[(f * M + r) * M + c] = (r == c) ? 1.0 : 0.0;
    bad |= ofc_mnmf_fit(F, T, M, N, K, x, P, lam, tp, va, 3, tr) != 0;
    (void)ofc_mnmf_loglik(F, T, M, N, K, x, P, lam, tp, va, llf);
    /* argument checks */
    bad |= ofc_fit(0, T, M, N, x, P, lam, v, 1, 0, NULL, 1) == 0;
    bad |= ofc_fit_blocks(F, T + 1, M, N, B, x, P, lam, vb, 1, 0, NULL, 1) == 0;
    free(x); free(P); free(lam); free(v); free(vb); free(y); free(tr); free(llf); free(Q); free(U);
    free(work); free(sig2); free(tp); free(va);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run(3, 12, 2, 3, 4, 2);
    bad |= run(2, 10, 3, 2, 2, 3);
    bad |= run(2, 8, 4, 6, 2, 2);
    bad |= run(1, 9, 8, 10, 3, 2);
    printf(bad ? "oracle driver: a call failed\n" : "oracle driver: ok\n");
    return bad;
}
