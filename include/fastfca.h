/*
 * fastfca.h -- C ABI of the MI355X (gfx950) FastFCA library.
 *
 * FastFCA (Ito, Ikeshita, Sawada, Nakatani, arXiv 2101.08563) fits, for every
 * frequency f of an M-channel STFT mixture x, jointly diagonalizable spatial
 * covariances R_n(f) = P(f)^{-H} diag(lambda_n(f)) P(f)^{-1} (Sec. IV-B,
 * eq:parametrizationFastFCA) and per-bin source powers v_n(t,f) by the IP+EM
 * iteration of Algorithm 1 (Sec. IV-E), then separates the N source images
 * with the multichannel Wiener filter in its decomposed form (Sec. IV-F,
 * eq:Doclo). The problem statement is Sec. II: estimate the source images
 * c_{f,t,n} given x_{f,t} and N, with M >= 2 and N >= 2.
 *
 * Notation: the paper's frequency index i is f here, its frame index j is t,
 * its decorrelation matrix W is P (column m is w_m), [L]_{mn} is
 * lambda[n][m] and [H]_{nj} is v[t][n].
 *
 * Conventions shared by every entry point
 *   - All array pointers are DEVICE pointers unless marked "host".
 *   - Layouts are dense row-major (C order), no padding:
 *       x      [F][T][M]     fastfca_c64   mixture STFT
 *       P      [F][M][M]     fastfca_c128  P[f][r][c]; column c is w_c, so the
 *                                          decorrelated mixture is
 *                                          y_m = sum_r conj(P[f][r][m]) x_r
 *       lambda [F][N][M]     float > 0     diag(Lambda_n(f)) = L[:,n]
 *       v      [F][T][N]     float > 0     h_{tn} at frequency f
 *       y      [N][F][T][M]  fastfca_c64   source images
 *   - The library copies x (and any initial parameters) into memory it owns,
 *     so the caller may free its buffers once fastfca_init returns. Output
 *     buffers are owned by the caller and written in stream order.
 *   - Every call returns a status (FASTFCA_OK or a negative error code); no
 *     call aborts or throws. fastfca_last_error() explains the last failure,
 *     including the failing mixture and frequency for numerical errors.
 *   - A context is bound to the HIP stream given at init; calls on one
 *     context must not overlap (not re-entrant). Separate contexts are
 *     independent.
 *   - Kernel-side numerical failures (non-finite values, singular IP
 *     systems) are recorded on the device and reported by the next
 *     synchronizing call: fastfca_sync, fastfca_loglik, fastfca_ll_trace.
 */
#ifndef FASTFCA_H
#define FASTFCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fastfca_ctx fastfca_ctx;

typedef struct { float re, im; } fastfca_c64;   /* == torch.complex64 element  */
typedef struct { double re, im; } fastfca_c128; /* == torch.complex128 element */

enum {
    FASTFCA_OK = 0,
    FASTFCA_E_ARG = -1,         /* invalid argument or shape                     */
    FASTFCA_E_NOMEM = -2,       /* device allocation failed                      */
    FASTFCA_E_HIP = -3,         /* HIP runtime error                             */
    FASTFCA_E_SINGULAR = -4,    /* IP system (eq:ip1) numerically singular       */
    FASTFCA_E_NONFINITE = -5,   /* NaN/Inf in input or in an iterate             */
    FASTFCA_E_STATE = -6,       /* call not valid in the context's state         */
    FASTFCA_E_UNSUPPORTED = -7  /* shape outside the compiled kernel families    */
};

/* Shape limits of the compiled kernels: 2 <= M <= FASTFCA_MAX_M,
 * 2 <= N <= FASTFCA_MAX_N, M <= T <= FASTFCA_MAX_T. Shapes with M <= 4,
 * N <= 8, T <= 2048 run with the whole frequency resident on chip; the rest
 * re-read x from device memory each iteration. */
#define FASTFCA_MAX_M 8
#define FASTFCA_MAX_N 12
#define FASTFCA_MAX_T 4096

/* One mixture of a batch (fastfca_init_batch). Pointer fields are device
 * pointers with the layouts above; P0/lambda0/v0 may be NULL (see init). */
typedef struct {
    const fastfca_c64 *x;
    int F, T, M, N;
    const fastfca_c128 *P0;
    const float *lambda0;
    const float *v0;
} fastfca_problem;

/*
 * fastfca_init -- create a context holding one mixture and its parameters.
 * Algorithm 1, "Initialize W, L, H": P0 == NULL sets P = I; lambda0/v0 ==
 * NULL draw lambda_nm = 0.5 + u and v_tn = (|x_t|^2/(MN) + d_f)(0.5 + u')
 * with d_f = 1e-6 mean_t |x_t|^2/(MN) and u, u' uniform on [0,1) from a
 * SplitMix64 counter stream keyed by `seed` (lambda: counter f*N*M + n*M + m;
 * v: counter 2^40 + (f*T + t)*N + n; u = (out >> 40) * 2^-24).
 * Validates shapes (E_ARG / E_UNSUPPORTED), x finiteness (E_NONFINITE) and
 * positivity of lambda0, v0 (E_ARG). hip_stream: a hipStream_t, or NULL for
 * the default stream. Synchronizes the stream before returning.
 * On failure *out is set to NULL and the error text is available from
 * fastfca_last_error(NULL).
 */
int fastfca_init(fastfca_ctx **out, const fastfca_c64 *x, int F, int T, int M, int N,
                 const fastfca_c128 *P0, const float *lambda0, const float *v0,
                 uint64_t seed, void *hip_stream);

/*
 * fastfca_init_batch -- a context holding B independent mixtures, each with
 * its own (F, T, M, N). probs is a HOST array of B descriptors whose pointer
 * fields are device pointers. All mixtures are iterated together by one
 * persistent launch per fastfca_em_step call. Initialization as in
 * fastfca_init; mixture b uses seed + b.
 */
int fastfca_init_batch(fastfca_ctx **out, int B, const fastfca_problem *probs,
                       uint64_t seed, void *hip_stream);

/*
 * fastfca_em_step -- run n_iter >= 1 iterations of Algorithm 1 (IP sweep over
 * m = 1..M using eq:wsampcov, eq:ip1, eq:ip2; U by eq:Udef; EM update of
 * L[:,n] then H[n,:] for n = 1..N in order) on every frequency of every
 * mixture. Asynchronous on the context's stream. The log-likelihood per TF
 * bin after each iteration (eq:negll, sign flipped, with the M ln(pi)
 * constant) is recorded for fastfca_ll_trace. Numerical failures freeze the
 * failing frequency and are reported by the next synchronizing call.
 */
int fastfca_em_step(fastfca_ctx *c, int n_iter);

/*
 * fastfca_sync -- wait for the context's stream; return the first recorded
 * numerical failure (E_SINGULAR / E_NONFINITE) or FASTFCA_OK.
 */
int fastfca_sync(fastfca_ctx *c);

/*
 * fastfca_loglik -- log-likelihood of the current parameters, per TF bin, of
 * mixture b (0 for a single-mixture context), in double precision
 * throughout (Sec. IV-D, eq:negll with the density constant of Sec. III-A):
 *   LL_f = ln|det P_f|^2 - (1/T) sum_{m,t} [ln pi + ln sigma^2_{mt} + U_{mt}/sigma^2_{mt}]
 *   *ll_per_bin (host) = (1/F) sum_f LL_f ;  ll_per_f (device [F] or NULL) = LL_f.
 * Synchronizes.
 */
int fastfca_loglik(fastfca_ctx *c, int b, double *ll_per_bin, double *ll_per_f);

/*
 * fastfca_ll_trace -- per-iteration LL per bin of mixture b recorded by the
 * last fastfca_em_step call: host array trace[n] for n < min(max_n, n_iter of
 * that call). Returns the number written (>= 0) or an error. Synchronizes.
 */
int fastfca_ll_trace(fastfca_ctx *c, int b, double *trace, int max_n);

/*
 * fastfca_mwf -- source images of mixture b by eq:Doclo:
 *   y_n(t,f) = P^{-H} diag_m( v_n lambda_{nm} / sigma^2_{mt} ) P^H x(t,f)
 * y: device [N][F][T][M] complex64 (caller-allocated). P^{-H} is formed in
 * double precision per frequency and applied in single precision.
 * Asynchronous; E_SINGULAR is reported by the next synchronizing call.
 */
int fastfca_mwf(fastfca_ctx *c, int b, fastfca_c64 *y);

/*
 * fastfca_get_params -- copy the current (P, lambda, v) of mixture b to
 * caller device buffers with the layouts above; any pointer may be NULL.
 * Stream-ordered (asynchronous).
 */
int fastfca_get_params(fastfca_ctx *c, int b, fastfca_c128 *P, float *lambda, float *v);

/*
 * fastfca_set_params -- overwrite the current (P, lambda, v) of mixture b
 * from caller device buffers (layouts above; any pointer may be NULL to keep
 * that parameter), i.e. re-run Algorithm 1's "Initialize W, L, H" with given
 * values: restarts, checkpoint resume, warm starts. Clears the recorded
 * failure state of the mixture. Values are not validated (lambda and v must
 * be finite and > 0). Stream-ordered (asynchronous).
 */
int fastfca_set_params(fastfca_ctx *c, int b, const fastfca_c128 *P, const float *lambda,
                       const float *v);

/* Shape of mixture b: writes F, T, M, N (host pointers; any may be NULL). */
int fastfca_shape(const fastfca_ctx *c, int b, int *F, int *T, int *M, int *N);

/* Number of mixtures held by the context. */
int fastfca_num_problems(const fastfca_ctx *c);

/*
 * fastfca_set_config -- override the launch configuration of every
 * subsequent fastfca_em_step: threads per workgroup (64..1024, multiple of
 * 64, or 0 = default) and bins per thread (2, 4, 8 or 16; 0 = default).
 * threads * bins_per_thread must cover the longest T of every (M,N) class and
 * may not exceed 2048 (4096 with 4 or 8 bins per thread for classes outside
 * the resident limits); E_ARG otherwise.
 */
int fastfca_set_config(fastfca_ctx *c, int threads, int bins_per_thread);

/*
 * fastfca_autotune -- time every admissible (threads, bins-per-thread) pair
 * for each (M,N) class of the context on a scratch copy of its state (the
 * context's parameters are left untouched), keep the fastest, and append the
 * result to the JSON-lines cache at cache_path (host string, may be NULL)
 * keyed by (gfx arch, M, N, T bucket). Synchronizes.
 */
int fastfca_autotune(fastfca_ctx *c, int n_iter, const char *cache_path);

/* Launch configuration in effect for the (M,N) class of mixture b. */
int fastfca_get_config(const fastfca_ctx *c, int b, int *threads, int *bins_per_thread);

/* Text of the last error of c (or of the last failed init when c is NULL). */
const char *fastfca_last_error(const fastfca_ctx *c);

/* Release every device buffer of c. c may be NULL. */
void fastfca_destroy(fastfca_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* FASTFCA_H */
