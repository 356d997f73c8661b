// C ABI of the warm-start network kernels (declared in include/fastfca.h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fastfca.h"
#include "internal.hpp"

namespace ffca {
hipError_t net_pack_weights(const float *W, int ldw, int Cout, int Cin, int KS, int Kp, int tf, uint16_t *Wb,
                            hipStream_t s);
hipError_t net_conv_fwd(const float *X, int S, int Cin, int T, const uint16_t *Wb, int Kp, int KS,
                        const float *bias, int Cout, float *Y, int mode, const float *Res, float *Pre,
                        hipStream_t s);
hipError_t net_conv_bwdw(const float *G, int S, int Cout, const float *X, int Cin, int T, int Kp, int KS,
                         float *dW, float *db, hipStream_t s);
hipError_t net_relu_grad(const float *G, const float *Pre, float *out, size_t n, hipStream_t s);
hipError_t net_mean_t(const float *H, int SC, int T, float *pooled, hipStream_t s);
hipError_t net_forward_fused(const float *feat, int S, int M, int T, int C, int L, int N,
                             const uint16_t *const *Wb, const float *const *b, int Kp0, const float *Wv, int ldv,
                             const float *bv, float *lv, float *part, float *pooled, hipStream_t s);
hipError_t net_mean_t_bwd(const float *dpooled, int SC, int T, float *dH, hipStream_t s);
hipError_t net_linear_fwd(const float *in, int S, int C, const float *Wl, const float *bl, int J, float *out,
                          hipStream_t s);
hipError_t net_linear_bwd(const float *in, int S, int C, const float *Wl, int J, const float *g, float *dWl,
                          float *dbl, float *din, hipStream_t s);
hipError_t net_pit_loss(const float *lv, const float *tv, const float *ll, const float *tl, int S, int N, int M,
                        int T, float wl, float *loss, int *perm, float *glv, float *gll, hipStream_t s);
hipError_t net_adamw(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                     float eps, float wd, int step, float gscale, hipStream_t s);
hipError_t net_features(const float2 *x, int F, int T, int M, float eps, double2 *P0, float *feat, hipStream_t s);
hipError_t net_targets(const double2 *P, const float *lam, const float *v, const double2 *P0, int F, int T, int M,
                       int N, float *tv, float *tl, hipStream_t s);
hipError_t net_apply_outputs(const float *lv, const float *ll, int F, int T, int M, int N, float *v, float *lam,
                             hipStream_t s);
}  // namespace ffca

using namespace ffca;

namespace {
thread_local std::string g_net_error;

int fin(hipError_t e, const char *what) {
    if (e == hipSuccess) return FASTFCA_OK;
    g_net_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorInvalidValue ? FASTFCA_E_ARG : FASTFCA_E_HIP;
}
int bad(const char *what) {
    g_net_error = std::string(what) + ": invalid arguments";
    return FASTFCA_E_ARG;
}
hipStream_t st(void *s) { return reinterpret_cast<hipStream_t>(s); }
}  // namespace

extern "C" {

const char *fastfca_net_last_error(void) { return g_net_error.c_str(); }

int fastfca_net_pack_weights(const float *W, int ldw, int Cout, int Cin, int ks, int Kp, int transpose_flip,
                             uint16_t *Wb, void *stream) {
    if (!W || !Wb || Cout < 1 || Cin < 1 || (ks != 1 && ks != 5) || Kp % 16 || ldw < Cin * ks ||
        Kp < (transpose_flip ? Cout : Cin) * ks)
        return bad("pack_weights");
    return fin(net_pack_weights(W, ldw, Cout, Cin, ks, Kp, transpose_flip, Wb, st(stream)), "pack_weights");
}

int fastfca_net_conv_fwd(const float *X, int S, int Cin, int T, const uint16_t *Wb, int Kp, int ks,
                         const float *bias, int Cout, float *Y, int mode, const float *Res, float *Pre,
                         void *stream) {
    if (!X || !Wb || !Y || S < 1 || T < 1 || Cin < 1 || Cout < 1 || mode < 0 || mode > 3 ||
        ((mode == 2 || mode == 3) && !Res))
        return bad("conv_fwd");
    return fin(net_conv_fwd(X, S, Cin, T, Wb, Kp, ks, bias, Cout, Y, mode, Res, Pre, st(stream)), "conv_fwd");
}

int fastfca_net_conv_bwd_weight(const float *G, int S, int Cout, const float *X, int Cin, int T, int Kp, int ks,
                                float *dW, float *db, void *stream) {
    if (!G || !X || !dW || S < 1 || T < 1 || Cin < 1 || Cout < 1) return bad("conv_bwd_weight");
    return fin(net_conv_bwdw(G, S, Cout, X, Cin, T, Kp, ks, dW, db, st(stream)), "conv_bwd_weight");
}

int fastfca_net_relu_grad(const float *G, const float *Pre, float *out, uint64_t n, void *stream) {
    if (!G || !Pre || !out) return bad("relu_grad");
    return fin(net_relu_grad(G, Pre, out, n, st(stream)), "relu_grad");
}

int fastfca_net_mean_t(const float *H, int SC, int T, float *pooled, void *stream) {
    if (!H || !pooled || SC < 1 || T < 1) return bad("mean_t");
    return fin(net_mean_t(H, SC, T, pooled, st(stream)), "mean_t");
}

int fastfca_net_mean_t_bwd(const float *dpooled, int SC, int T, float *dH, void *stream) {
    if (!dpooled || !dH || SC < 1 || T < 1) return bad("mean_t_bwd");
    return fin(net_mean_t_bwd(dpooled, SC, T, dH, st(stream)), "mean_t_bwd");
}

int fastfca_net_forward_fused(const float *feat, int S, int M, int T, int C, int L, int N,
                              const uint16_t *const *Wb, const float *const *b, int Kp0, const float *Wv, int ldv,
                              const float *bv, float *lv, float *part, float *pooled, void *stream) {
    if (!feat || !Wb || !b || !Wv || !bv || !lv || !part || !pooled) return bad("forward_fused");
    return fin(net_forward_fused(feat, S, M, T, C, L, N, Wb, b, Kp0, Wv, ldv, bv, lv, part, pooled, st(stream)),
               "forward_fused");
}

int fastfca_net_linear_fwd(const float *in, int S, int C, const float *Wl, const float *bl, int J, float *out,
                           void *stream) {
    if (!in || !Wl || !bl || !out || S < 1 || C < 1 || J < 1) return bad("linear_fwd");
    return fin(net_linear_fwd(in, S, C, Wl, bl, J, out, st(stream)), "linear_fwd");
}

int fastfca_net_linear_bwd(const float *in, int S, int C, const float *Wl, int J, const float *g, float *dWl,
                           float *dbl, float *din, void *stream) {
    if (!in || !Wl || !g || !dWl || !dbl || !din || S < 1 || C < 1 || J < 1) return bad("linear_bwd");
    return fin(net_linear_bwd(in, S, C, Wl, J, g, dWl, dbl, din, st(stream)), "linear_bwd");
}

int fastfca_net_pit_loss(const float *lv, const float *tv, const float *ll, const float *tl, int S, int N, int M,
                         int T, float wl, float *loss, int *perm, float *glv, float *gll, void *stream) {
    if (!lv || !tv || !ll || !tl || !loss || S < 1 || N < 1 || N > 4 || M < 1 || T < 1) return bad("pit_loss");
    return fin(net_pit_loss(lv, tv, ll, tl, S, N, M, T, wl, loss, perm, glv, gll, st(stream)), "pit_loss");
}

int fastfca_net_adamw(float *p, const float *g, float *m, float *v, uint64_t n, float lr, float beta1,
                      float beta2, float eps, float weight_decay, int step, float grad_scale, void *stream) {
    if (!p || !g || !m || !v || step < 1) return bad("adamw");
    return fin(net_adamw(p, g, m, v, n, lr, beta1, beta2, eps, weight_decay, step, grad_scale, st(stream)), "adamw");
}

int fastfca_ws_features(const fastfca_c64 *x, int F, int T, int M, float eps, fastfca_c128 *P0, float *feat,
                        void *stream) {
    if (!x || !P0 || !feat || F < 1 || T < 1 || M < 1 || M > 4) return bad("features");
    return fin(net_features(reinterpret_cast<const float2 *>(x), F, T, M, eps, reinterpret_cast<double2 *>(P0),
                            feat, st(stream)),
               "features");
}

int fastfca_ws_targets(const fastfca_c128 *P, const float *lambda, const float *v, const fastfca_c128 *P0, int F,
                       int T, int M, int N, float *tv, float *tl, void *stream) {
    if (!P || !lambda || !v || !P0 || !tv || !tl || F < 1 || T < 1 || M < 1 || M > 4 || N < 1) return bad("targets");
    return fin(net_targets(reinterpret_cast<const double2 *>(P), lambda, v, reinterpret_cast<const double2 *>(P0),
                           F, T, M, N, tv, tl, st(stream)),
               "targets");
}

int fastfca_ws_apply(const float *lv, const float *ll, int F, int T, int M, int N, float *v, float *lambda,
                     void *stream) {
    if (!lv || !ll || !v || !lambda || F < 1 || T < 1 || M < 1 || N < 1) return bad("apply");
    return fin(net_apply_outputs(lv, ll, F, T, M, N, v, lambda, st(stream)), "apply");
}

}  // extern "C"
