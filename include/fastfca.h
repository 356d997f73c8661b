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
    FASTFCA_E_UNSUPPORTED = -7, /* shape outside the compiled kernel families    */
    FASTFCA_E_DECREASE = -8     /* log-likelihood fell between two iterations   */
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
 * fastfca_init_blocks -- a context holding one mixture fitted with the
 * piecewise stationary model (Sec. VI, eq:negllpws): the T frames of x are
 * split into J = T / block_len blocks of block_len consecutive frames that
 * share the source powers h, and Algorithms 1 and 2 run on the block
 * covariances Xhat_j = (1/block_len) sum_b x x^H in place of x_t x_t^H
 * (Q_m = (1/J) sum_j Xhat_j / sigma^2_mj, U_mj = w_m^H Xhat_j w_m).
 * T must be a positive multiple of block_len and J >= M; block_len = 1
 * gives the frame model through this path. v0 (and the v of get/set_params)
 * is [F][J][N]; fastfca_shape reports T = J; fastfca_mwf writes all T
 * frames, each with its block's h. Runs the on-chip kernels: M <= 4, N <= 8,
 * J <= 2048 (E_UNSUPPORTED otherwise). Otherwise as fastfca_init.
 */
int fastfca_init_blocks(fastfca_ctx **out, const fastfca_c64 *x, int F, int T, int M, int N,
                        int block_len, const fastfca_c128 *P0, const float *lambda0,
                        const float *v0, uint64_t seed, void *hip_stream);

/* Frames per block of mixture b of a fastfca_init_blocks context; 0 for a
 * frame context; E_ARG for a bad index. */
int fastfca_block_length(const fastfca_ctx *c, int b);

/*
 * fastfca_mnmf_init -- a context fitting FastMNMF (Sec. V, "FastMNMF:
 * Full-band Extension of FastFCA", and its appendix): the source powers are
 * an NMF over frequency and time, h_{ijn} = sum_k t_{ikn} v_{jkn}
 * (eq:NMFconst2), and eq:FastMNMFcost is minimized by IP for every P(f)
 * (eq:ip1, eq:ip2) and by the multiplicative MM rule for Lambda, then T, then
 * V, each rule theta <- theta sqrt(sum phi U / sigma^4 / sum phi / sigma^2)
 * for the coefficient phi of theta in sigma^2.
 *   x       device [F][T][M] complex64 (copied)
 *   K       NMF bases per source, 1..32
 *   P0      device [F][M][M] complex128, or NULL for P = I
 *   lambda0 device [F][N][M] > 0 (required)
 *   t0      device [F][K][N] > 0, spectral patterns t_{ikn} (required)
 *   v0      device [T][K][N] > 0, activations v_{jkn} (required)
 * M <= 4, N <= 6, T <= 2048 (E_UNSUPPORTED otherwise). fastfca_em_step runs
 * IP+MM iterations (one per-frequency launch and one pass over frames per
 * iteration); fastfca_loglik, fastfca_ll_trace and fastfca_mwf use the
 * current h, which fastfca_get_params returns as v [F][T][N]. set_config,
 * autotune and set_algorithm return E_STATE / E_UNSUPPORTED. An activation
 * that reaches zero or a non-finite value is reported as E_NONFINITE.
 */
int fastfca_mnmf_init(fastfca_ctx **out, const fastfca_c64 *x, int F, int T, int M, int N, int K,
                      const fastfca_c128 *P0, const float *lambda0, const float *t0,
                      const float *v0, void *hip_stream);

/* FastMNMF factors (device pointers, any may be NULL): P [F][M][M],
 * lambda [F][N][M], t [F][K][N], v [T][K][N]. E_STATE for other contexts. */
int fastfca_mnmf_get_params(fastfca_ctx *c, fastfca_c128 *P, float *lambda, float *t, float *v);
int fastfca_mnmf_set_params(fastfca_ctx *c, const fastfca_c128 *P, const float *lambda,
                            const float *t, const float *v);

/*
 * fastfca_em_step -- run n_iter >= 1 iterations of Algorithm 1 (IP sweep over
 * m = 1..M using eq:wsampcov, eq:ip1, eq:ip2; U by eq:Udef; EM update of
 * L[:,n] then H[n,:] for n = 1..N in order) on every frequency of every
 * mixture. Asynchronous on the context's stream. The log-likelihood per TF
 * bin after each iteration (eq:negll, sign flipped, with the M ln(pi)
 * constant) is recorded for fastfca_ll_trace. Numerical failures freeze the
 * failing frequency and are reported by the next synchronizing call.
 * Contexts of one (M, N, T) class are launched directly (one launch, plus
 * those of the tail split); batches of several classes, the persistent
 * schedule and FastMNMF replay a HIP graph captured once per n_iter.
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
 * Precision: the per-bin terms ln sigma^2 and U / sigma^2 of eq:negll are
 * formed in single precision inside the EM kernels, from the single
 * precision per-bin statistics, and summed in double precision in a fixed
 * order; ln|det P|^2 is double precision. fastfca_loglik evaluates the same
 * quantity entirely in double precision; on the tested mixtures the trace
 * agrees with the double precision likelihood within 1e-6 nats per bin for
 * M <= 4 and within 2e-6 for the wide kernels' M up to 8 (the single
 * precision logarithms of the per-bin terms).
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

/* Update of L and H inside each iteration of fastfca_em_step. */
enum {
    FASTFCA_ALGO_EM = 0, /* Algorithm 1 (IP+EM): sources updated in order, the default */
    FASTFCA_ALGO_MM = 1  /* Algorithm 2 (IP+MM): multiplicative square-root rules, L then H */
};

/*
 * fastfca_set_algorithm -- choose the L/H update of later fastfca_em_step
 * calls (Sec. IV-E: Algorithm 1 or Algorithm 2; the IP update of P and the
 * log-likelihood are shared), for every shape fastfca_init accepts (the
 * resident and the wide kernel families). E_UNSUPPORTED for a FastMNMF
 * context, whose updates are MM by construction.
 */
int fastfca_set_algorithm(fastfca_ctx *c, int algo);

/*
 * fastfca_set_ll_alarm -- tolerance of the likelihood alarm of later
 * fastfca_em_step calls. Algorithms 1 and 2 never lower the log-likelihood
 * (Sec. III-C, Sec. IV-E); a frequency whose recorded LL per bin falls by
 * more than tol between two iterations of one call is stopped there with
 * FASTFCA_E_DECREASE (reported, with the frequency, by the next
 * synchronizing call), as a sign that the arithmetic has broken down.
 * Default 1e-3; +INFINITY disables the alarm; NaN is E_ARG.
 */
int fastfca_set_ll_alarm(fastfca_ctx *c, double tol);

/*
 * fastfca_set_tail_split -- schedule of a context whose items form one class
 * (a single mixture, or a batch of equal shapes) in later fastfca_em_step
 * calls. When the frequencies all fit on the GPU at once but their number is
 * not a multiple of the compute-unit count, r = n mod CUs of the CUs carry
 * one workgroup more than the rest for the whole call. The split runs the
 * first n - r frequencies as one launch and the last r in consecutive
 * launches of about n_iter / blocks iterations each, on a side stream and at
 * the highest wave priority, so that the extra load is spread over several
 * CUs. The iterations are the same (Algorithm 1 or 2, in order, state kept
 * exactly between launches): results and the LL trace are bitwise those of
 * the unsplit schedule; the likelihood alarm compares consecutive iterations
 * within each launch.
 *   blocks  -1 (default): automatic, min(8, n_iter / 10) blocks when the
 *           shape qualifies and that makes at least 2; 0: never split;
 *           1..1024: that many blocks (at most n_iter) whenever the shape
 *           qualifies. The shape qualifies with one round of workgroups
 *           when 1 <= r <= CUs / 4 and the extra workgroup adds a wave to
 *           a SIMD of its CU (otherwise the CUs carrying it are no slower),
 *           and with several rounds when the last round holds at most a
 *           quarter of the slots.
 * Errors: FASTFCA_E_ARG for a NULL context or blocks outside -1..1024.
 */
int fastfca_set_tail_split(fastfca_ctx *c, int blocks);

/* Schedule of a batch context's fastfca_em_step. */
enum {
    FASTFCA_SCHEDULE_CLASSES = 0,    /* one launch per (M, N, T-bucket) class, workgroups sized to T */
    FASTFCA_SCHEDULE_PERSISTENT = 1  /* one persistent launch over a longest-first work queue */
};

/*
 * fastfca_set_schedule -- choose how a batch context iterates (both give the
 * same results up to the launch shape's summation order). fastfca_autotune
 * times both and keeps the faster. E_UNSUPPORTED for the persistent schedule
 * on a single mixture or a batch with classes outside its compiled set.
 */
int fastfca_set_schedule(fastfca_ctx *c, int schedule);

/* Launch configuration in effect for the (M,N) class of mixture b. */
int fastfca_get_config(const fastfca_ctx *c, int b, int *threads, int *bins_per_thread);

/*
 * fastfca_synth_mixture -- draw a seeded synthetic mixture x [F][T][M]
 * (device, complex64, caller-allocated) from the FCA generative model of
 * Sec. III-A: c_n ~ N_c(0, v_n R_n), x = sum_n c_n (eq:summodel), with
 * v_n = W_n H_n of rank `rank` (Exp(1) factors) and R_n(f) = a a^H +
 * diffuse I, a_m = exp(i theta) with theta uniform. Counter-based
 * (SplitMix64) so any mixture is reproducible from (seed, shape). A data
 * utility for benchmarks and training sets, not part of the method.
 * Allocates and frees a small workspace; synchronizes the stream.
 * Limits: 1 <= M <= 8, N >= 1, rank >= 1.
 */
int fastfca_synth_mixture(fastfca_c64 *x, int F, int T, int M, int N, int rank, float diffuse,
                          uint64_t seed, void *hip_stream);

/* Text of the last error of c (or of the last failed init when c is NULL). */
const char *fastfca_last_error(const fastfca_ctx *c);

/* Release every device buffer of c. c may be NULL. */
void fastfca_destroy(fastfca_ctx *c);

/* ====================================================================
 * Learned warm start (not in the paper; the paper lists initialization
 * robustness and convergence acceleration as future work, Sec. VIII).
 * A 1-D convolutional network over time, applied to every frequency with
 * shared weights, maps whitened log-powers to initial lambda and v; the
 * IP+EM iteration then refines them. All pointers are device pointers; all
 * calls are asynchronous on the given stream; they return FASTFCA_OK,
 * FASTFCA_E_ARG (bad shape/argument) or FASTFCA_E_HIP, with text in
 * fastfca_net_last_error().
 *
 * Tensors: activations float [S][C][T] (S sequences, i.e. frequencies,
 * C <= 64 channels); a convolution with kernel size ks in {1, 5} and zero
 * "same" padding uses weights float [Cout][Cin][ks] packed to bfloat16
 * [Cout][Kp], Kp = Cin*ks rounded up to a multiple of 16 (<= 320), for the
 * 16x16x16 bf16 MFMA with float accumulation.
 * ==================================================================== */

/* Text of the last error of the network entry points. */
const char *fastfca_net_last_error(void);

/* Pack float weights W (row co at W + co*ldw holding entries ci*ks + k,
 * ldw >= Cin*ks) into the bf16 GEMM operand Wb[Cout][Kp], column order
 * k-major: Wb[co][k*Cin + ci] = W[co][ci*ks + k]; with transpose_flip != 0
 * into the operand of the data-gradient convolution, Wb[ci][k*Cout + co] =
 * W[co][ci*ks + ks-1-k] (Kp >= Cout*ks, Cin rows). */
int fastfca_net_pack_weights(const float *W, int ldw, int Cout, int Cin, int ks, int Kp, int transpose_flip,
                             uint16_t *Wb, void *stream);

/* Y[s][co][t] = epilogue(pre), pre = bias[co] + sum_{ci,k} W[co][ci][k] X[s][ci][t+k-ks/2]
 * (X zero outside [0,T)); mode 0: Y = pre, 1: relu(pre), 2: Res + relu(pre),
 * 3: Res + pre. bias may be NULL (zero); Pre (optional) receives pre.
 * Res and Y are [S][Cout][T]; Y may alias Res. */
int fastfca_net_conv_fwd(const float *X, int S, int Cin, int T, const uint16_t *Wb, int Kp, int ks,
                         const float *bias, int Cout, float *Y, int mode, const float *Res, float *Pre,
                         void *stream);

/* Weight and bias gradients of the convolution, ACCUMULATED (+=) into float
 * dW (row co at dW + co*Kp, entry ci*ks + k: the layout of the float master
 * packed by fastfca_net_pack_weights with ldw = Kp) and db[Cout] (may be NULL):
 * dW += sum_{s,t} G[s][co][t] X[s][ci][t+k-ks/2]. Float atomics: the
 * summation order is not fixed. */
int fastfca_net_conv_bwd_weight(const float *G, int S, int Cout, const float *X, int Cin, int T, int Kp,
                                int ks, float *dW, float *db, void *stream);

/* out[i] = G[i] if Pre[i] > 0 else 0, i < n. */
int fastfca_net_relu_grad(const float *G, const float *Pre, float *out, uint64_t n, void *stream);

/* pooled[i] = (1/T) sum_t H[i][t], i < SC (SC = S*C rows of length T). */
int fastfca_net_mean_t(const float *H, int SC, int T, float *pooled, void *stream);

/* dH[i][t] += dpooled[i] / T. */
int fastfca_net_mean_t_bwd(const float *dpooled, int SC, int T, float *dH, void *stream);

/*
 * fastfca_net_forward_fused -- inference forward of the whole network in one
 * launch: the kernel-5 input layer, L residual kernel-5 layers and the 1x1
 * head, for tiles of 64 frames with the activations in LDS (the same BF16
 * operands and FP32 accumulation as fastfca_net_conv_fwd; the head in FP32).
 *   feat    device [S][M][T] float32 features, M <= 4
 *   Wb, b   HOST arrays of L + 1 device pointers: packed BF16 weights of the
 *           kernel-5 layers (layer 0 [C][Kp0], Kp0 = 16 or 32, >= 5 M;
 *           layers 1..L [C][5 C]) and their FP32 biases [C]
 *   Wv, bv  device FP32 head weights [N][ldv] (entry c of row n, ldv >= C)
 *           and biases [N], N <= 8
 *   lv      device [S][N][T] output (log v before the positivity map)
 *   part    device scratch, S * ceil(T / 64) * C floats
 *   pooled  device [S][C] output, the mean over t of the last layer
 * C a multiple of 16 up to 64, L <= 8. E_ARG on other shapes or NULL
 * pointers. Asynchronous on hip_stream. For inference only: no activation is
 * kept for the backward pass.
 */
int fastfca_net_forward_fused(const float *feat, int S, int M, int T, int C, int L, int N,
                              const uint16_t *const *Wb, const float *const *b, int Kp0,
                              const float *Wv, int ldv, const float *bv, float *lv, float *part,
                              float *pooled, void *stream);

/* out[s][j] = bl[j] + sum_c Wl[j][c] in[s][c]. */
int fastfca_net_linear_fwd(const float *in, int S, int C, const float *Wl, const float *bl, int J,
                           float *out, void *stream);

/* Gradients of linear_fwd: dWl[j][c] += sum_s g[s][j] in[s][c],
 * dbl[j] += sum_s g[s][j], din[s][c] = sum_j Wl[j][c] g[s][j]. */
int fastfca_net_linear_bwd(const float *in, int S, int C, const float *Wl, int J, const float *g,
                           float *dWl, float *dbl, float *din, void *stream);

/* Permutation-invariant loss per sequence s (N <= 4 sources):
 *   loss[s] = min over orders pi of
 *     mean_{n,t} (lv[s][pi(n)][t] - tv[s][n][t])^2 + wl * mean_{n,m} (ll[s][pi(n)][m] - tl[s][n][m])^2
 * (orders enumerated lexicographically, first minimum kept); perm [S][N]
 * (optional) receives pi; glv [S][N][T], gll [S][N][M] (optional) receive the
 * gradient of loss[s] through the minimizing order. */
int fastfca_net_pit_loss(const float *lv, const float *tv, const float *ll, const float *tl, int S, int N,
                         int M, int T, float wl, float *loss, int *perm, float *glv, float *gll,
                         void *stream);

/* AdamW step (decoupled weight decay) on n parameters: m, v moments; the
 * gradient is scaled by grad_scale first; step >= 1 sets the bias
 * corrections 1 - beta^step. */
int fastfca_net_adamw(float *p, const float *g, float *m, float *v, uint64_t n, float lr, float beta1,
                      float beta2, float eps, float weight_decay, int step, float grad_scale, void *stream);

/* Warm-start features of one mixture x [F][T][M] (M <= 4): per frequency
 * C = (1/T) sum_t x_t x_t^H, P0 = C^{-1/2} (double precision, coupled
 * Newton-Schulz) written to P0 [F][M][M], and
 * feat[f][m][t] = ln(|(P0^H x_t)_m|^2 + eps) minus its mean over t. */
int fastfca_ws_features(const fastfca_c64 *x, int F, int T, int M, float eps, fastfca_c128 *P0, float *feat,
                        void *stream);

/* Training targets from a fit (P, lambda, v) and the whitening P0 (M <= 4):
 * each source is scaled so that tr R_n = M (R_n = P^{-H} diag(lambda_n) P^{-1},
 * the trace normalization of the paper's SCM error, eq:Rerror); then
 * tv[f][n][t] = ln(c_n v[f][t][n]) and tl[f][n][m] = ln [P0^H (R_n/c_n) P0]_{mm},
 * c_n = tr R_n / M. */
int fastfca_ws_targets(const fastfca_c128 *P, const float *lambda, const float *v, const fastfca_c128 *P0,
                       int F, int T, int M, int N, float *tv, float *tl, void *stream);

/* Network outputs to initial parameters: v[f][t][n] = exp(lv[f][n][t]),
 * lambda[f][n][m] = exp(ll[f][n][m]) (arguments clamped to [-60, 60]). */
int fastfca_ws_apply(const float *lv, const float *ll, int F, int T, int M, int N, float *v, float *lambda,
                     void *stream);

/*
 * The trained warm-start network as fastfca_warmstart consumes it: the
 * operands of fastfca_net_forward_fused plus the lambda head. Every pointer
 * is a device pointer owned by the caller except Wb and b, HOST arrays of
 * L + 1 device pointers.
 *   M, N     microphones and sources (must match the mixture), N <= 8, M <= 4
 *   C, L     channels (a multiple of 16 up to 64) and residual layers (<= 8)
 *   Wb, b    packed BF16 kernel-5 weights and FP32 biases of layers 0..L
 *   Kp0      row length of the packed layer-0 weights (16 or 32, >= 5 M)
 *   Wv, ldv  FP32 head weights [N][ldv] (ldv >= C); bv its biases [N]
 *   Wl, bl   FP32 lambda head [N*M][C] and biases [N*M]
 */
typedef struct {
    int M, N, C, L;
    const uint16_t *const *Wb;
    const float *const *b;
    int Kp0;
    const float *Wv;
    int ldv;
    const float *bv;
    const float *Wl;
    const float *bl;
} fastfca_net;

/*
 * fastfca_warmstart -- replace the current start of mixture b by a learned
 * warm start, judged by the method itself (the paper names initialization
 * and convergence acceleration as future work, Sec. VIII; the IP+EM
 * iteration that follows is the refiner, the fallback and the judge):
 *   1. P <- P0 = C_f^{-1/2} and the features (fastfca_ws_features);
 *   2. net != NULL: the network (fastfca_net_forward_fused, the lambda head)
 *      and lambda = exp(ll), v = exp(lv) (fastfca_ws_apply);
 *      net == NULL: the whitening-only start lambda = 1,
 *      v_tn = (1/(M N)) sum_m |(P0^H x_t)_m|^2;
 *   3. judge, per frequency (every frequency is its own problem, Sec. II):
 *      the new start is kept where its log-likelihood (eq:negll, double
 *      precision, as fastfca_loglik) is finite and not below that of the
 *      start it replaces; elsewhere that start is restored bit for bit.
 * Frame-model contexts (fastfca_init, fastfca_init_batch) with M <= 4 only:
 * E_STATE for block and FastMNMF contexts, E_ARG for a network whose shape
 * does not match. Asynchronous on the context's stream unless n_taken
 * (host, may be NULL) is given: then it synchronizes and stores the number
 * of frequencies that kept the new start. Clears the mixture's recorded
 * failure state. Allocates its workspace (features, activations, the saved
 * start) on the first call for a mixture size and keeps it with the context.
 */
int fastfca_warmstart(fastfca_ctx *c, int b, const fastfca_net *net, int *n_taken);

/*
 * fastfca_warmstart_race -- the warm start judged by a race instead of by
 * the starting likelihood. The current start of mixture b (A) and the new
 * one (B: the network's, or with net == NULL the whitening-only start, as in
 * fastfca_warmstart) both run race_iters >= 1 iterations of the context's
 * algorithm (Algorithm 1, or 2 after fastfca_set_algorithm), side by side in
 * one launch over 2F frequencies; then each frequency keeps the state with
 * the higher log-likelihood per bin after the race (eq:negll, from the
 * fused trace; a start whose run stopped with an error loses). The mixture's
 * state is then race_iters iterations on from its better start, frequency by
 * frequency; later fastfca_em_step calls continue from there. The starts
 * often converge to different local optima of a frequency, so keeping the
 * better one can raise the likelihood reached faster than either start.
 *   n_taken  host int or NULL: the number of frequencies that kept B (the
 *            call then synchronizes).
 * Workspace as fastfca_warmstart, plus 16 F race_iters bytes of traces.
 * Errors: as fastfca_warmstart; FASTFCA_E_ARG for race_iters < 1. The
 * context's own trace (fastfca_ll_trace) is not written.
 */
int fastfca_warmstart_race(fastfca_ctx *c, int b, const fastfca_net *net, int race_iters, int *n_taken);

/* ====================================================================
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * ==================================================================== */

/* Bytes of the fixed device array fastfca_fit_noalloc works in (one per GPU,
 * held from the first call on that GPU until the process ends). */
#define FASTFCA_NOALLOC_SCRATCH_BYTES (8u << 20)

/*
 * fastfca_fit_noalloc -- n_iter >= 1 iterations of Algorithm 1 (the same
 * kernels and launch shape as fastfca_em_step on a context made by
 * fastfca_init) on one mixture held in the caller's device buffers, with no
 * device allocation, free, copy or memset:
 *   x        [F][T][M] complex64, read in place (must be finite)
 *   P        [F][M][M] complex128, lambda [F][N][M], v [F][T][N]: the start
 *            on entry, updated in place (lambda, v > 0)
 *   status   [F] int, output: 0, or FASTFCA_E_SINGULAR / FASTFCA_E_NONFINITE /
 *            FASTFCA_E_DECREASE (the likelihood alarm at its default
 *            tolerance, see fastfca_set_ll_alarm) for a frequency whose
 *            iteration failed (its state is left where it stopped)
 *   ll_trace [F][n_iter] double, output, or NULL: LL per bin of frequency f
 *            after each iteration (eq:negll; the library's trace terms)
 * The per-frequency work table, ln|det P|^2 and (when ll_trace is NULL) the
 * trace live in the library's fixed device array: 256-byte aligned parts of
 * 64 F, 8 F and 8 F n_iter bytes must fit in FASTFCA_NOALLOC_SCRATCH_BYTES
 * (E_ARG otherwise; e.g. F = 513 allows n_iter <= 1900 without ll_trace).
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (on different streams or host threads) race. Shapes as fastfca_init
 * (E_ARG, E_UNSUPPORTED). Asynchronous on hip_stream (NULL: the default
 * stream); the error text of a rejected call is in fastfca_last_error(NULL).
 */
int fastfca_fit_noalloc(const fastfca_c64 *x, int F, int T, int M, int N, fastfca_c128 *P, float *lambda,
                        float *v, int n_iter, int *status, double *ll_trace, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FASTFCA_H */
