// Host runtime of the FastFCA library: context and buffer management,
// validation, kernel dispatch, hipGraph replay of em_step, and the launch
// configuration autotuner. Implements include/fastfca.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/fastfca.h"
#include "internal.hpp"
#include "mnmf.hpp"

namespace ffca {
hipError_t launch_ldet(const WorkItem *items, int n_items, int M, double *ldet, hipStream_t s);
hipError_t launch_loglik_terms(const WorkItem *items, int n_items, int M, const double *ldet,
                               double *ll_f, hipStream_t s);
hipError_t launch_mwf_bins(const WorkItem *items, int F, int T, int M, float2 *y, hipStream_t s);
hipError_t launch_synth(float2 *x, int F, int T, int M, int N, int K, float delta, uint64_t seed,
                        float *W, float2 *C, hipStream_t s);
hipError_t launch_ws_whitened(const float2 *x, const double2 *P, float *lam, float *v, int F, int T, int M, int N,
                              hipStream_t s);
hipError_t launch_ws_select(const double *ll_old, const double *ll_new, double2 *P, float *lam, float *v,
                            const double2 *P_old, const float *lam_old, const float *v_old, int F, int T, int M,
                            int N, int *n_taken, hipStream_t s, int *status = nullptr,
                            const int *status_old = nullptr, double *ldet = nullptr,
                            const double *ldet_old = nullptr);
hipError_t launch_race_ll(const double *trace, int K, const int *st_b, const int *st_a, double *ll_b, double *ll_a,
                          int F, hipStream_t s);
hipError_t net_features(const float2 *x, int F, int T, int M, float eps, double2 *P0, float *feat, hipStream_t s);
hipError_t net_forward_fused(const float *feat, int S, int M, int T, int C, int L, int N,
                             const uint16_t *const *Wb, const float *const *b, int Kp0, const float *Wv, int ldv,
                             const float *bv, float *lv, float *part, float *pooled, hipStream_t s);
hipError_t net_linear_fwd(const float *in, int S, int C, const float *Wl, const float *bl, int J, float *out,
                          hipStream_t s);
hipError_t net_apply_outputs(const float *lv, const float *ll, int F, int T, int M, int N, float *v, float *lam,
                             hipStream_t s);
}  // namespace ffca

using namespace ffca;

namespace {

thread_local std::string g_init_error;
// Error text of fastfca_fit_noalloc: a fixed buffer, so that a rejected call
// allocates nothing either. fastfca_last_error(NULL) returns the newer of the
// two messages.
thread_local char g_noalloc_error[256];
thread_local bool g_noalloc_error_newer = false;

struct Problem {
    int F = 0, T = 0, M = 0, N = 0;  // T: bins of the iteration (frames, or blocks)
    int B = 1;                       // frames per block (piecewise stationary model)
    bool blocks = false;             // bins are blocks with covariances in z
    float2 *x = nullptr;             // [F][T*B][M]
    float *z = nullptr;              // [F][T][M*M] block covariances (blocks only)
    float *v = nullptr;
    float *lam = nullptr;
    double2 *P = nullptr;
    double *ldet = nullptr;
    double *llf = nullptr;
    WorkItem *items = nullptr;  // this mixture's items in frequency order
    int item0 = 0;  // index of frequency 0 in the context's item array
};

struct ClassCfg {
    int M, N, Tmax;
    int bucket = 0;     // batches: workgroup size of a 4-bins-per-thread launch for T (0: one class per (M, N))
    bool cov = false;   // bins carry block covariances (piecewise stationary model)
    bool wide = false;  // wide family (x re-read per iteration) instead of resident
    int threads = 0, bpt = 0;
    std::vector<int> items;  // item indices of this class, in launch order
};

// Workspace of fastfca_warmstart, sized for the largest mixture seen. Each
// buffer has its capacity in elements beside it.
template <typename T>
struct WsBuf {
    T *p = nullptr;
    size_t cap = 0;
};
struct WsScratch {
    WsBuf<float> feat;      // [F][M][T] features
    WsBuf<float> lv;        // [F][N][T] network log v
    WsBuf<float> part;      // fused forward's per-tile sums
    WsBuf<float> pooled;    // [F][C]
    WsBuf<float> ll;        // [F][N*M] network log lambda
    WsBuf<double2> P_old;   // the start being replaced
    WsBuf<float> lam_old;
    WsBuf<float> v_old;
    WsBuf<double> ll_old;   // [F] per-frequency LL of the replaced start
    WsBuf<double> ll_new;   // [F] per-frequency LL of the new start
    WsBuf<int> taken;       // frequencies that kept the new start
    // fastfca_warmstart_race: both starts' traces, the copy's ln|det P|^2 and
    // status, and the work table of the 2F frequencies that race
    WsBuf<double> race_trace;
    WsBuf<double> race_ldet;
    WsBuf<int> race_status;
    WsBuf<WorkItem> race_items;
    std::vector<WorkItem> race_host;  // the table as last uploaded
};

// FastMNMF state (fastfca_mnmf_init): NMF factors and the V-rule scratch.
struct MnmfState {
    int K = 0, threads = 0, bpt = 0;
    float *tp = nullptr;    // [F][K][N]
    float *va = nullptr;    // [K][N][T] (the ABI's [T][K][N] transposed)
    float *G = nullptr, *E = nullptr;  // [F][T][N]
    float *part = nullptr;  // [chunks][2][K][T][N]
    int *vflag = nullptr;
};

}  // namespace

// Default tolerance of the likelihood alarm (nats per bin, per frequency,
// between two iterations of one call): far above the single precision
// noise of the per-iteration trace, far below any real decrease.
constexpr double kDefaultLLAlarm = 1e-3;

struct fastfca_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // side streams (default priority) over which the class launches of a
    // batch are spread so that one class fills the tail of another; forked
    // from and joined back into `stream` with events (also inside a capture)
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[kSide] = {nullptr, nullptr, nullptr};
    std::vector<Problem> probs;
    std::vector<WorkItem> h_items;
    WorkItem *d_items = nullptr;      // in launch order (grouped by class)
    std::vector<int> item_pos;        // problem item index -> position in d_items
    int *d_status = nullptr;
    double *d_trace = nullptr;
    int trace_cap = 0;
    int last_n_iter = 0;
    int *d_queue = nullptr;
    std::vector<ClassCfg> classes;
    std::vector<int> class_first;     // first position of each class in d_items
    bool persistent = false;          // batch: one persistent launch
    int p_threads = 0, p_bpt = 0, p_grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_n_iter = -1;
    int algo = kAlgoEM;
    double ll_alarm = kDefaultLLAlarm;  // fastfca_set_ll_alarm
    int tail_split = -1;              // fastfca_set_tail_split: -1 automatic, 0 off, k > 0 blocks
    int ncu = 0;                      // compute units of the device
    MnmfState *mn = nullptr;          // FastMNMF context
    WsScratch ws;                     // fastfca_warmstart workspace
    std::string err;
    char arch[64] = {0};
};

namespace {

int set_err(fastfca_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
    } else {
        g_init_error = buf;
        g_noalloc_error_newer = false;
    }
    return code;
}

#define HIPCHK(c, expr)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return set_err((c), FASTFCA_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
int dalloc(fastfca_ctx *c, T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return FASTFCA_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return set_err(c, FASTFCA_E_NOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                       hipGetErrorString(e));
    }
    return FASTFCA_OK;
}

// (Re)allocate one workspace buffer to hold at least n elements.
template <typename T>
int ws_reserve(fastfca_ctx *c, WsBuf<T> &b, size_t n) {
    if (n <= b.cap && b.p) return FASTFCA_OK;
    hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    int rc = dalloc(c, &b.p, n);
    if (rc == FASTFCA_OK) b.cap = n;
    return rc;
}

void free_problem(Problem &p) {
    hipFree(p.x);
    hipFree(p.z);
    hipFree(p.v);
    hipFree(p.lam);
    hipFree(p.P);
    hipFree(p.ldet);
    hipFree(p.llf);
    hipFree(p.items);
    p = Problem{};
}

void drop_graph(fastfca_ctx *c) {
    if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_n_iter = -1;
}

// Smallest workgroup (multiple of 64) holding T bins at bpt bins per thread,
// or 0 if it exceeds the family's limit (threads * bpt <= cap).
int threads_for(int T, int bpt, int cap = kResidentBins) {
    int th = ((T + bpt - 1) / bpt + 63) / 64 * 64;
    if (th < 64) th = 64;
    return th * bpt <= cap ? th : 0;
}

// Default (threads, bins per thread) of a class; M = 0: the persistent
// kernel's shape for a batch (four bins per thread first).
bool pick_default(int M, int N, int Tmax, int &threads, int &bpt) {
    // From sweeps on gfx950 over M = 2, 3, 4, N = M + 1 .. 8 and T = 200..2000
    // (513 frequencies, 100 iterations, every shape that fits):
    //   T <= 256:        four (at M = 2 from 129 frames two, in two
    //                    wavefronts: 3-4 % faster on the 250-block
    //                    piecewise model);
    //   256 < T <= 512:  eight, one wavefront (up to 6 % faster than four,
    //                    ties at N = 8), except M = 3, N = 5, whose
    //                    eight-bin instance spills (3.5 % slower);
    //   512 < T <= 1024: four;
    //   T > 1024:        eight (M = 2, 3: 25-30 % faster than four; M = 4:
    //                    1-4 %).
    // Two bins per thread was never the fastest beyond 256 frames.
    if (M == 2 && threads_for(Tmax, 4) == 64 && threads_for(Tmax, 2) == 128) {
        threads = 128;
        bpt = 2;
        return true;
    }
    const bool mid = threads_for(Tmax, 4) == 128 && !(M == 3 && N == 5);
    const bool eight = M > 0 && (Tmax > 1024 || mid);
    for (int b : {eight ? 8 : 4, eight ? 4 : 8, 2}) {
        const int th = threads_for(Tmax, b);
        if (th) {
            threads = th;
            bpt = b;
            return true;
        }
    }
    return false;
}

// Kernel family of an (M, N, Tmax) class: resident when its bins fit on chip
// next to x, wide otherwise.
bool use_resident(int M, int N, int Tmax) {
    return M <= 4 && N <= 8 && Tmax <= kResidentBins && em_supported(M, N, 4);
}

// Default launch shape of a class.
bool pick_class(ClassCfg &cc) {
    if (cc.cov) {  // block model: resident family only
        cc.wide = false;
        return use_resident(cc.M, cc.N, cc.Tmax) && pick_default(cc.M, cc.N, cc.Tmax, cc.threads, cc.bpt);
    }
    cc.wide = !use_resident(cc.M, cc.N, cc.Tmax);
    if (!cc.wide) return pick_default(cc.M, cc.N, cc.Tmax, cc.threads, cc.bpt);
    // wide family: four bins per thread when at most 512 threads hold the
    // frames (T <= 2048), 1.2-1.6x faster than eight (sweep on gfx950 at
    // M = 5, 6, 8 and T = 300..2000); eight beyond
    const int th4 = threads_for(cc.Tmax, 4, kWideMaxT);
    if (th4 && th4 <= wide_max_threads(4) && em_wide_supported(cc.M, cc.N, 4)) {
        cc.bpt = 4;
        cc.threads = th4;
        return true;
    }
    cc.bpt = 8;
    cc.threads = threads_for(cc.Tmax, 8, kWideMaxT);  // at most 512 (kWideMaxThreads)
    return cc.threads != 0 && em_wide_supported(cc.M, cc.N, 8);
}


int validate_shape(fastfca_ctx *c, int F, int T, int M, int N) {
    if (F < 1 || T < 1 || M < 2 || N < 2)
        return set_err(c, FASTFCA_E_ARG, "invalid shape F=%d T=%d M=%d N=%d (need F,T>=1, M,N>=2)",
                       F, T, M, N);
    if (T < M)
        return set_err(c, FASTFCA_E_ARG, "T=%d < M=%d: the weighted covariances are singular", T, M);
    if (M > FASTFCA_MAX_M || N > FASTFCA_MAX_N || T > FASTFCA_MAX_T)
        return set_err(c, FASTFCA_E_UNSUPPORTED, "shape M=%d N=%d T=%d beyond the compiled limits", M,
                       N, T);
    return FASTFCA_OK;
}

// Builds classes, item order, device item array. Assumes problem buffers exist.
int build_items(fastfca_ctx *c) {
    // A class is one (M, N) kernel instantiation; in a batch, mixtures are
    // further grouped by T so that each class launch has a workgroup sized to
    // its frames (a mixture with T = 200 does not run in a 512-thread block).
    std::map<std::tuple<int, int, int>, int> cls_of;
    auto key_of = [&](const Problem &p) {
        const int bucket = (c->probs.size() > 1 && !p.blocks && use_resident(p.M, p.N, p.T)) ? threads_for(p.T, 4) : 0;
        return std::make_tuple(p.M, p.N + (p.blocks ? 1000 : 0), bucket);
    };
    c->classes.clear();
    for (auto &p : c->probs) {
        auto key = key_of(p);
        if (!cls_of.count(key)) {
            cls_of[key] = static_cast<int>(c->classes.size());
            ClassCfg cc;
            cc.M = p.M;
            cc.N = p.N;
            cc.cov = p.blocks;
            cc.bucket = std::get<2>(key);
            cc.Tmax = 0;
            c->classes.push_back(cc);
        }
        auto &cc = c->classes[cls_of[key]];
        cc.Tmax = std::max(cc.Tmax, p.T);
    }
    int total = 0;
    for (auto &p : c->probs) {
        p.item0 = total;
        total += p.F;
    }
    c->h_items.assign(total, WorkItem{});
    for (size_t b = 0; b < c->probs.size(); ++b) {
        auto &p = c->probs[b];
        const int cls = cls_of[key_of(p)];
        for (int f = 0; f < p.F; ++f) {
            WorkItem w{};
            w.x = p.x + static_cast<size_t>(f) * p.T * p.B * p.M;
            w.z = p.blocks ? p.z + static_cast<size_t>(f) * p.T * p.M * p.M : nullptr;
            w.B = p.B;
            w.Tx = p.T * p.B;
            w.v = p.v + static_cast<size_t>(f) * p.T * p.N;
            w.lam = p.lam + static_cast<size_t>(f) * p.N * p.M;
            w.P = p.P + static_cast<size_t>(f) * p.M * p.M;
            w.ldet = p.ldet + f;
            w.T = p.T;
            w.M = p.M;
            w.N = p.N;
            w.cls = cls;
            c->h_items[p.item0 + f] = w;
            c->classes[cls].items.push_back(p.item0 + f);
        }
    }
    // longest items first inside each class (list scheduling)
    for (auto &cc : c->classes)
        std::stable_sort(cc.items.begin(), cc.items.end(), [&](int a, int b) {
            return c->h_items[a].T > c->h_items[b].T;
        });
    for (auto &cc : c->classes) {
        if (!pick_class(cc))
            return set_err(c, FASTFCA_E_UNSUPPORTED, "no compiled kernel for M=%d N=%d T=%d%s", cc.M,
                           cc.N, cc.Tmax,
                           cc.cov ? " (the block model runs M<=4, N<=8, at most 2048 blocks)" : "");
    }
    int rc;
    if ((rc = dalloc(c, &c->d_status, total)) != FASTFCA_OK) return rc;
    if ((rc = dalloc(c, &c->d_items, total)) != FASTFCA_OK) return rc;
    if ((rc = dalloc(c, &c->d_queue, 1)) != FASTFCA_OK) return rc;
    HIPCHK(c, launch_fill_int(c->d_status, total, ST_OK, c->stream));
    return FASTFCA_OK;
}

// (Re)allocates the LL trace and uploads the item array in launch order.
int upload_items(fastfca_ctx *c, int n_iter) {
    const int total = static_cast<int>(c->h_items.size());
    if (n_iter > c->trace_cap || !c->d_trace) {
        int cap = std::max(n_iter, 128);
        hipFree(c->d_trace);
        c->d_trace = nullptr;
        int rc = dalloc(c, &c->d_trace, static_cast<size_t>(cap) * total);
        if (rc != FASTFCA_OK) return rc;
        c->trace_cap = cap;
        drop_graph(c);
    }
    std::vector<WorkItem> ordered;
    ordered.reserve(total);
    c->item_pos.assign(total, 0);
    c->class_first.clear();
    auto push = [&](int i) {
        WorkItem w = c->h_items[i];
        w.ll_trace = c->d_trace + static_cast<size_t>(i) * c->trace_cap;
        w.status = c->d_status + i;
        c->item_pos[i] = static_cast<int>(ordered.size());
        ordered.push_back(w);
    };
    if (c->persistent) {
        // one queue over every item, costliest first (longest-processing-time
        // list scheduling); cost ~ T * (M + N)
        std::vector<int> order(total);
        for (int i = 0; i < total; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const auto &A = c->h_items[a], &B = c->h_items[b];
            return static_cast<long>(A.T) * (A.M + A.N) > static_cast<long>(B.T) * (B.M + B.N);
        });
        for (int i : order) push(i);
    } else {
        for (auto &cc : c->classes) {
            c->class_first.push_back(static_cast<int>(ordered.size()));
            for (int i : cc.items) push(i);
        }
    }
    HIPCHK(c, hipMemcpyAsync(c->d_items, ordered.data(), sizeof(WorkItem) * total,
                             hipMemcpyHostToDevice, c->stream));
    for (auto &p : c->probs) {
        if (!p.items) {
            int rc = dalloc(c, &p.items, p.F);
            if (rc != FASTFCA_OK) return rc;
        }
        std::vector<WorkItem> own(p.F);
        for (int f = 0; f < p.F; ++f) {
            own[f] = c->h_items[p.item0 + f];
            own[f].ll_trace = c->d_trace + static_cast<size_t>(p.item0 + f) * c->trace_cap;
            own[f].status = c->d_status + p.item0 + f;
        }
        HIPCHK(c, hipMemcpyAsync(p.items, own.data(), sizeof(WorkItem) * p.F, hipMemcpyHostToDevice,
                                 c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FASTFCA_OK;
}

int alloc_problem(fastfca_ctx *c, Problem &p) {
    int rc;
    const size_t F = p.F, T = p.T, M = p.M, N = p.N;
    if ((rc = dalloc(c, &p.x, F * T * p.B * M)) != FASTFCA_OK) return rc;
    if (p.blocks && (rc = dalloc(c, &p.z, F * T * M * M)) != FASTFCA_OK) return rc;
    if ((rc = dalloc(c, &p.v, F * T * N)) != FASTFCA_OK) return rc;
    if ((rc = dalloc(c, &p.lam, F * N * M)) != FASTFCA_OK) return rc;
    if ((rc = dalloc(c, &p.P, F * M * M)) != FASTFCA_OK) return rc;
    if ((rc = dalloc(c, &p.ldet, F)) != FASTFCA_OK) return rc;
    if ((rc = dalloc(c, &p.llf, F)) != FASTFCA_OK) return rc;
    return FASTFCA_OK;
}

int init_problem(fastfca_ctx *c, Problem &p, const fastfca_problem &d, uint64_t seed, int b) {
    const size_t F = p.F, T = p.T, M = p.M, N = p.N, Tx = static_cast<size_t>(p.T) * p.B;
    HIPCHK(c, hipMemcpyAsync(p.x, d.x, sizeof(float2) * F * Tx * M, hipMemcpyDeviceToDevice,
                             c->stream));
    int *flag = nullptr;
    int rc = dalloc(c, &flag, 3);
    if (rc != FASTFCA_OK) return rc;
    int hflag[3] = {0, 0, 0};
    hipError_t e = hipMemcpyAsync(flag, hflag, sizeof hflag, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_check_finite_x(p.x, F * Tx * M, flag, c->stream);
    if (e == hipSuccess && d.lambda0) e = launch_check_positive(d.lambda0, F * N * M, flag + 1, c->stream);
    if (e == hipSuccess && d.v0) e = launch_check_positive(d.v0, F * T * N, flag + 2, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    hipFree(flag);
    if (e != hipSuccess) return set_err(c, FASTFCA_E_HIP, "validation failed: %s", hipGetErrorString(e));
    if (hflag[0]) return set_err(c, FASTFCA_E_NONFINITE, "mixture %d: x holds NaN or Inf", b);
    if (hflag[1]) return set_err(c, FASTFCA_E_ARG, "mixture %d: lambda0 must be finite and > 0", b);
    if (hflag[2]) return set_err(c, FASTFCA_E_ARG, "mixture %d: v0 must be finite and > 0", b);
    if (d.P0)
        HIPCHK(c, hipMemcpyAsync(p.P, d.P0, sizeof(double2) * F * M * M, hipMemcpyDeviceToDevice,
                                 c->stream));
    else
        HIPCHK(c, launch_identity_P(p.P, p.F, p.M, c->stream));
    if (d.lambda0)
        HIPCHK(c, hipMemcpyAsync(p.lam, d.lambda0, sizeof(float) * F * N * M,
                                 hipMemcpyDeviceToDevice, c->stream));
    if (d.v0)
        HIPCHK(c, hipMemcpyAsync(p.v, d.v0, sizeof(float) * F * T * N, hipMemcpyDeviceToDevice,
                                 c->stream));
    if (p.blocks) HIPCHK(c, launch_block_cov(p.x, p.z, p.F, p.T, p.B, p.M, c->stream));
    if (!d.lambda0 || !d.v0)
        HIPCHK(c, launch_seeded_init(p.x, p.z, p.lam, p.v, p.F, p.T, p.M, p.N, seed, !d.lambda0, !d.v0,
                                     c->stream));
    return FASTFCA_OK;
}

// block_len > 0: one mixture fitted with the piecewise stationary model,
// blocks of block_len frames (probs[0].T frames in x).
int create(fastfca_ctx **out, int B, const fastfca_problem *probs, uint64_t seed, void *stream,
           int block_len = 0) {
    if (!out) return set_err(nullptr, FASTFCA_E_ARG, "out is NULL");
    *out = nullptr;
    if (B < 1 || !probs) return set_err(nullptr, FASTFCA_E_ARG, "need B >= 1 problems");
    if (block_len > 0) {
        if (B != 1) return set_err(nullptr, FASTFCA_E_ARG, "the block model takes one mixture");
        if (probs[0].T < block_len || probs[0].T % block_len != 0)
            return set_err(nullptr, FASTFCA_E_ARG, "T=%d frames is not a positive multiple of the block length %d",
                           probs[0].T, block_len);
    }
    for (int b = 0; b < B; ++b) {
        const auto &d = probs[b];
        int rc = validate_shape(nullptr, d.F, block_len > 0 ? d.T / block_len : d.T, d.M, d.N);
        if (rc != FASTFCA_OK) {
            g_init_error = "mixture " + std::to_string(b) + ": " + g_init_error;
            return rc;
        }
        if (!d.x) return set_err(nullptr, FASTFCA_E_ARG, "mixture %d: x is NULL", b);
    }
    auto *c = new fastfca_ctx();
    c->stream = reinterpret_cast<hipStream_t>(stream);
    hipGetDevice(&c->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess)
        snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
    c->probs.resize(B);
    int rc = FASTFCA_OK;
    for (int b = 0; b < B && rc == FASTFCA_OK; ++b) {
        auto &p = c->probs[b];
        p.F = probs[b].F;
        p.T = probs[b].T;
        p.M = probs[b].M;
        p.N = probs[b].N;
        if (block_len > 0) {
            p.blocks = true;
            p.B = block_len;
            p.T = probs[b].T / block_len;
        }
        rc = alloc_problem(c, p);
        if (rc == FASTFCA_OK) rc = init_problem(c, p, probs[b], seed + static_cast<uint64_t>(b), b);
    }
    if (rc == FASTFCA_OK) rc = build_items(c);
    if (rc == FASTFCA_OK) {
        // side streams: the class schedule of a batch (the default; the
        // persistent queue is kept ready as the alternative the autotuner
        // times) and the tail split of a single class
        if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
            c->ncu = 0;
        {
            bool ok = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
            for (int q = 0; q < fastfca_ctx::kSide && ok; ++q)
                ok = hipStreamCreateWithFlags(&c->side[q], hipStreamNonBlocking) == hipSuccess &&
                     hipEventCreateWithFlags(&c->join[q], hipEventDisableTiming) == hipSuccess;
            if (!ok) rc = set_err(c, FASTFCA_E_HIP, "could not create the side streams");
        }
        c->persistent = B > 1;
        if (c->persistent) {
            // one persistent launch: the widest class sets the block shape
            int Tmax = 0;
            bool ok = true;
            for (auto &cc : c->classes) {
                Tmax = std::max(Tmax, cc.Tmax);
                ok = ok && !cc.wide && persistent_supported(cc.M, cc.N);
            }
            if (!ok || !pick_default(0, 0, Tmax, c->p_threads, c->p_bpt)) {
                c->persistent = false;
                c->p_threads = 0;
            }
            if (c->persistent) {
                if (c->p_bpt == 2) c->p_bpt = 4;
                int ncu = 256;
                if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) !=
                    hipSuccess)
                    ncu = 256;
                c->p_grid = ncu * std::max(1, 2048 / c->p_threads);
            }
        }
        c->persistent = false;
        if (rc == FASTFCA_OK) rc = upload_items(c, 128);
    }
    if (rc == FASTFCA_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = set_err(c, FASTFCA_E_HIP, "init: %s", hipGetErrorString(e));
    }
    if (rc != FASTFCA_OK) {
        g_init_error = c->err;
        fastfca_destroy(c);
        return rc;
    }
    *out = c;
    return FASTFCA_OK;
}

int record_mnmf(fastfca_ctx *c, int n_iter) {
    auto &p = c->probs[0];
    auto &mn = *c->mn;
    MnmfLaunch a{};
    a.x = p.x;
    a.P = p.P;
    a.lam = p.lam;
    a.tp = mn.tp;
    a.va = mn.va;
    a.G = mn.G;
    a.E = mn.E;
    a.ll_trace = c->d_trace;
    a.cap = c->trace_cap;
    a.ldet = p.ldet;
    a.status = c->d_status;
    a.F = p.F;
    a.T = p.T;
    a.K = mn.K;
    for (int it = 0; it <= n_iter; ++it) {
        a.iter = it;
        a.ll_only = it == n_iter;
        HIPCHK(c, launch_mnmf_freq(p.M, p.N, mn.bpt, mn.threads, a, c->stream));
        if (it < n_iter)
            HIPCHK(c, launch_mnmf_v(mn.G, mn.E, mn.tp, mn.part, mn.va, p.F, p.T, p.N, mn.K, kMnmfFChunk, mn.vflag,
                                    c->stream));
    }
    // the frame-model h for the likelihood, MWF and parameter calls
    HIPCHK(c, launch_mnmf_h(mn.tp, mn.va, p.v, p.F, p.T, p.N, mn.K, c->stream));
    return FASTFCA_OK;
}

// Tail split of a single class. Its n workgroups take the CUs in rounds of
// S = CUs x (workgroups a CU holds at once). When they all fit in one round
// (n <= S), a remainder of r = n mod CUs makes r CUs carry one workgroup more
// than the others for the whole call; with several rounds, a last partial
// round of r = n mod S workgroups runs alone. Either way the call waits for
// those r frequencies. The split runs the first n - r items as one launch
// and the last r in `blocks` consecutive launches of about n_iter / blocks
// iterations each, on a side stream, at the highest wave priority: each block
// lands on whichever CU has room (with several rounds, in the gaps as the
// rounds drain), so the extra load is spread thin over several CUs, and the
// priority keeps the r frequencies' own chain of iterations as fast as the
// rest. The state between blocks (P in double precision, L, H) is stored
// exactly, so the results are bitwise those of one launch; the likelihood
// alarm compares consecutive iterations within a block.
constexpr int kSimdsPerCu = 4;

struct TailPlan {
    int r = 0;       // items in the tail (0: no split)
    int blocks = 0;  // launches the tail's iterations are cut into
};

TailPlan tail_plan(const fastfca_ctx *c, const ClassCfg &cc, int n_iter) {
    TailPlan t;
    const int n = static_cast<int>(cc.items.size());
    const int C = c->ncu;
    if (c->tail_split == 0 || C <= 0 || !c->side[0]) return t;
    if (!(cc.wide ? em_wide_tail_supported(cc.M, cc.N, cc.bpt) : em_tail_supported(cc.M, cc.N, cc.bpt, cc.cov)))
        return t;
    const int cap = cc.wide ? em_wide_blocks_per_cu(cc.M, cc.N, cc.bpt, cc.threads)
                            : em_blocks_per_cu(cc.M, cc.N, cc.bpt, cc.threads, cc.cov);
    if (cap < 1) return t;
    const long S = static_cast<long>(C) * cap;
    int r;
    if (n <= S) {
        r = n % C;
        if (n < C || r < 1 || r > C / 4) return t;
        // the extra workgroup must add a wave to some SIMD of its CU, or the
        // CUs that carry it are no slower than the rest (short frames: a
        // workgroup of one wave per frequency)
        const int W = (cc.threads + 63) / 64, base = n / C;
        if ((base + 1) * W <= kSimdsPerCu * ((base * W + kSimdsPerCu - 1) / kSimdsPerCu)) return t;
    } else {
        r = static_cast<int>(n % S);
        if (r < 1 || r > S / 4) return t;
    }
    int k = c->tail_split > 0 ? c->tail_split : std::min(8, n_iter / 10);
    k = std::min(k, n_iter);
    if (k < 2) return t;
    t.r = r;
    t.blocks = k;
    return t;
}

hipError_t launch_class(const ClassCfg &cc, const EmLaunch &a, int grid, hipStream_t st) {
    return cc.wide ? launch_em_wide(cc.M, cc.N, cc.bpt, cc.threads, a, grid, st)
                   : launch_em(cc.M, cc.N, cc.bpt, cc.threads, a, grid, st, cc.cov);
}

int record_em(fastfca_ctx *c, int n_iter) {
    if (c->mn) return record_mnmf(c, n_iter);
    if (c->persistent) {
        HIPCHK(c, launch_fill_int(c->d_queue, 1, 0, c->stream));
        EmLaunch a{c->d_items, static_cast<int>(c->h_items.size()), n_iter, c->d_queue, c->algo, c->ll_alarm};
        HIPCHK(c, launch_em_persistent(a, c->p_threads, c->p_bpt, c->p_grid, c->stream));
        return FASTFCA_OK;
    }
    // classes in decreasing total cost, spread round-robin over the context
    // stream and the side streams when there are several
    const int ncls = static_cast<int>(c->classes.size());
    std::vector<int> order(ncls);
    for (int k = 0; k < ncls; ++k) order[k] = k;
    auto cost = [&](int k) {
        const auto &cc = c->classes[k];
        return static_cast<double>(cc.items.size()) * cc.Tmax * (cc.M + cc.N);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    if (ncls == 1) {
        const auto &cc = c->classes[0];
        const TailPlan tp = tail_plan(c, cc, n_iter);
        if (tp.r > 0) {
            const int n = static_cast<int>(cc.items.size());
            const WorkItem *items = c->d_items + c->class_first[0];
            HIPCHK(c, hipEventRecord(c->fork, c->stream));
            HIPCHK(c, hipStreamWaitEvent(c->side[0], c->fork, 0));
            EmLaunch a{items, n - tp.r, n_iter, nullptr, c->algo, c->ll_alarm, 0, 0};
            HIPCHK(c, launch_class(cc, a, n - tp.r, c->stream));
            for (int j = 0; j < tp.blocks; ++j) {
                const int i0 = static_cast<int>(static_cast<long>(n_iter) * j / tp.blocks);
                const int i1 = static_cast<int>(static_cast<long>(n_iter) * (j + 1) / tp.blocks);
                EmLaunch b{items + (n - tp.r), tp.r, i1 - i0, nullptr, c->algo, c->ll_alarm, i0, 1};
                HIPCHK(c, launch_class(cc, b, tp.r, c->side[0]));
            }
            HIPCHK(c, hipEventRecord(c->join[0], c->side[0]));
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->join[0], 0));
            return FASTFCA_OK;
        }
    }
    const int nstreams = (ncls > 1 && c->side[0]) ? 1 + fastfca_ctx::kSide : 1;
    if (nstreams > 1) {
        HIPCHK(c, hipEventRecord(c->fork, c->stream));
        for (int q = 0; q < fastfca_ctx::kSide; ++q) HIPCHK(c, hipStreamWaitEvent(c->side[q], c->fork, 0));
    }
    for (int r = 0; r < ncls; ++r) {
        const int k = order[r];
        const auto &cc = c->classes[k];
        hipStream_t st = (r % nstreams) == 0 ? c->stream : c->side[(r % nstreams) - 1];
        EmLaunch a{c->d_items + c->class_first[k], static_cast<int>(cc.items.size()), n_iter,
                   nullptr, c->algo, c->ll_alarm};
        if (cc.wide)
            HIPCHK(c, launch_em_wide(cc.M, cc.N, cc.bpt, cc.threads, a,
                                     static_cast<int>(cc.items.size()), st));
        else
            HIPCHK(c, launch_em(cc.M, cc.N, cc.bpt, cc.threads, a, static_cast<int>(cc.items.size()),
                                st, cc.cov));
    }
    if (nstreams > 1) {
        for (int q = 0; q < fastfca_ctx::kSide; ++q) {
            HIPCHK(c, hipEventRecord(c->join[q], c->side[q]));
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->join[q], 0));
        }
    }
    return FASTFCA_OK;
}

int check_status(fastfca_ctx *c) {
    const int total = static_cast<int>(c->h_items.size());
    std::vector<int> st(total);
    int vflag = 0;
    HIPCHK(c, hipMemcpyAsync(st.data(), c->d_status, sizeof(int) * total, hipMemcpyDeviceToHost,
                             c->stream));
    if (c->mn)
        HIPCHK(c, hipMemcpyAsync(&vflag, c->mn->vflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (vflag) return set_err(c, FASTFCA_E_NONFINITE, "FastMNMF: an activation v became zero or non-finite");
    for (size_t b = 0; b < c->probs.size(); ++b) {
        const auto &p = c->probs[b];
        for (int f = 0; f < p.F; ++f) {
            const int s = st[p.item0 + f];
            if (s != ST_OK)
                return set_err(c, s, "mixture %zu frequency %d: %s", b, f,
                               s == ST_SINGULAR   ? "IP system numerically singular"
                               : s == ST_DECREASE ? "log-likelihood decreased between two iterations"
                                                  : "non-finite value in an iterate");
        }
    }
    return FASTFCA_OK;
}

bool valid_problem(fastfca_ctx *c, int b) { return c && b >= 0 && b < static_cast<int>(c->probs.size()); }

}  // namespace

// ====================================================================== ABI
// ------------------------------------------------------------------ allocation-free fit
// Device memory of fastfca_fit_noalloc: the per-frequency work table, ln|det P|^2
// and (when the caller passes no trace buffer) the likelihood trace. One copy
// per GPU, kept until the process ends; host code reaches it only through the
// per-device address taken with hipGetSymbolAddress (the array's name is a
// host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[FASTFCA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoallocMaxDevices = 64;
void *g_scratch_ptr[kNoallocMaxDevices] = {};
std::mutex g_scratch_mu;

int noalloc_err(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_noalloc_error, sizeof g_noalloc_error, fmt, ap);
    va_end(ap);
    g_noalloc_error_newer = true;
    return code;
}

// Address of the scratch array on the current device, taken once per device.
int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return noalloc_err(FASTFCA_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kNoallocMaxDevices) return noalloc_err(FASTFCA_E_HIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return noalloc_err(FASTFCA_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                               hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FASTFCA_OK;
}

// Work table of one mixture held in caller buffers; also clears its status.
__global__ void noalloc_items_kernel(WorkItem *items, const float2 *x, double2 *P, float *lam, float *v,
                                     double *trace, int trace_stride, double *ldet, int *status, int F, int T, int M,
                                     int N) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    WorkItem w{};
    w.x = x + static_cast<size_t>(f) * T * M;
    w.z = nullptr;
    w.v = v + static_cast<size_t>(f) * T * N;
    w.lam = lam + static_cast<size_t>(f) * N * M;
    w.P = P + static_cast<size_t>(f) * M * M;
    w.ll_trace = trace + static_cast<size_t>(f) * trace_stride;
    w.ldet = ldet + f;
    w.status = status + f;
    w.T = T;
    w.M = M;
    w.N = N;
    w.B = 1;
    w.Tx = T;
    w.cls = 0;
    items[f] = w;
    status[f] = ST_OK;
}

constexpr size_t align256(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

extern "C" {

int fastfca_init(fastfca_ctx **out, const fastfca_c64 *x, int F, int T, int M, int N,
                 const fastfca_c128 *P0, const float *lambda0, const float *v0, uint64_t seed,
                 void *hip_stream) {
    fastfca_problem d{x, F, T, M, N, P0, lambda0, v0};
    return create(out, 1, &d, seed, hip_stream);
}

int fastfca_init_batch(fastfca_ctx **out, int B, const fastfca_problem *probs, uint64_t seed,
                       void *hip_stream) {
    return create(out, B, probs, seed, hip_stream);
}

int fastfca_init_blocks(fastfca_ctx **out, const fastfca_c64 *x, int F, int T, int M, int N,
                        int block_len, const fastfca_c128 *P0, const float *lambda0, const float *v0,
                        uint64_t seed, void *hip_stream) {
    if (block_len < 1) return set_err(nullptr, FASTFCA_E_ARG, "block length must be >= 1");
    fastfca_problem d{x, F, T, M, N, P0, lambda0, v0};
    return create(out, 1, &d, seed, hip_stream, block_len);
}

int fastfca_mnmf_init(fastfca_ctx **out, const fastfca_c64 *x, int F, int T, int M, int N, int K,
                      const fastfca_c128 *P0, const float *lambda0, const float *t0, const float *v0,
                      void *hip_stream) {
    if (!out) return set_err(nullptr, FASTFCA_E_ARG, "out is NULL");
    *out = nullptr;
    if (!lambda0 || !t0 || !v0) return set_err(nullptr, FASTFCA_E_ARG, "FastMNMF needs lambda0, t0 and v0");
    if (K < 1 || K > kMnmfKMax) return set_err(nullptr, FASTFCA_E_ARG, "K=%d outside 1..%d", K, kMnmfKMax);
    if (M < 2 || M > 4 || N < 2 || N > kMnmfNMax || T > kResidentBins)
        return set_err(nullptr, FASTFCA_E_UNSUPPORTED, "FastMNMF runs M<=4, N<=%d, T<=%d (M=%d N=%d T=%d)",
                       kMnmfNMax, kResidentBins, M, N, T);
    fastfca_problem d{x, F, T, M, N, P0, lambda0, nullptr};
    // frame-model context for x, P, Lambda, h (= v) and the likelihood/MWF kernels
    int rc = create(out, 1, &d, 0, hip_stream);
    if (rc != FASTFCA_OK) return rc;
    fastfca_ctx *c = *out;
    auto *mn = new MnmfState();
    c->mn = mn;
    mn->K = K;
    mn->bpt = N >= 6 ? 8 : 4;
    mn->threads = threads_for(T, mn->bpt);
    const size_t Fs = F, Ts = T, Ns = N, Ks = K;
    const size_t nchunk = (F + kMnmfFChunk - 1) / kMnmfFChunk;
    int *flag = nullptr;
    int hflag[2] = {0, 0};
    hipError_t e = hipSuccess;
    if ((rc = dalloc(c, &mn->tp, Fs * Ks * Ns)) == FASTFCA_OK && (rc = dalloc(c, &mn->va, Ts * Ks * Ns)) == FASTFCA_OK &&
        (rc = dalloc(c, &mn->G, Fs * Ts * Ns)) == FASTFCA_OK && (rc = dalloc(c, &mn->E, Fs * Ts * Ns)) == FASTFCA_OK &&
        (rc = dalloc(c, &mn->part, nchunk * 2 * Ks * Ts * Ns)) == FASTFCA_OK &&
        (rc = dalloc(c, &mn->vflag, 1)) == FASTFCA_OK && (rc = dalloc(c, &flag, 2)) == FASTFCA_OK) {
        e = hipMemcpyAsync(mn->tp, t0, sizeof(float) * Fs * Ks * Ns, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = launch_transpose(v0, mn->va, T, K * N, c->stream);
        if (e == hipSuccess) e = launch_fill_int(mn->vflag, 1, 0, c->stream);
        if (e == hipSuccess) e = launch_fill_int(flag, 2, 0, c->stream);
        if (e == hipSuccess) e = launch_check_positive(mn->tp, Fs * Ks * Ns, flag, c->stream);
        if (e == hipSuccess) e = launch_check_positive(mn->va, Ts * Ks * Ns, flag + 1, c->stream);
        if (e == hipSuccess) e = launch_mnmf_h(mn->tp, mn->va, c->probs[0].v, F, T, N, K, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = set_err(c, FASTFCA_E_HIP, "FastMNMF init: %s", hipGetErrorString(e));
        else if (hflag[0] || hflag[1]) rc = set_err(c, FASTFCA_E_ARG, "t0 and v0 must be finite and > 0");
    }
    hipFree(flag);
    if (rc != FASTFCA_OK) {
        g_init_error = c->err;
        fastfca_destroy(c);
        *out = nullptr;
    }
    return rc;
}

int fastfca_mnmf_get_params(fastfca_ctx *c, fastfca_c128 *P, float *lambda, float *t, float *v) {
    if (!c || !c->mn) return c ? set_err(c, FASTFCA_E_STATE, "not a FastMNMF context") : FASTFCA_E_ARG;
    auto &p = c->probs[0];
    const size_t F = p.F, T = p.T, M = p.M, N = p.N, K = c->mn->K;
    if (P) HIPCHK(c, hipMemcpyAsync(P, p.P, sizeof(double2) * F * M * M, hipMemcpyDeviceToDevice, c->stream));
    if (lambda)
        HIPCHK(c, hipMemcpyAsync(lambda, p.lam, sizeof(float) * F * N * M, hipMemcpyDeviceToDevice, c->stream));
    if (t) HIPCHK(c, hipMemcpyAsync(t, c->mn->tp, sizeof(float) * F * K * N, hipMemcpyDeviceToDevice, c->stream));
    if (v) HIPCHK(c, launch_transpose(c->mn->va, v, static_cast<int>(K * N), static_cast<int>(T), c->stream));
    return FASTFCA_OK;
}

int fastfca_mnmf_set_params(fastfca_ctx *c, const fastfca_c128 *P, const float *lambda, const float *t,
                            const float *v) {
    if (!c || !c->mn) return c ? set_err(c, FASTFCA_E_STATE, "not a FastMNMF context") : FASTFCA_E_ARG;
    auto &p = c->probs[0];
    const size_t F = p.F, T = p.T, M = p.M, N = p.N, K = c->mn->K;
    if (P) HIPCHK(c, hipMemcpyAsync(p.P, P, sizeof(double2) * F * M * M, hipMemcpyDeviceToDevice, c->stream));
    if (lambda)
        HIPCHK(c, hipMemcpyAsync(p.lam, lambda, sizeof(float) * F * N * M, hipMemcpyDeviceToDevice, c->stream));
    if (t) HIPCHK(c, hipMemcpyAsync(c->mn->tp, t, sizeof(float) * F * K * N, hipMemcpyDeviceToDevice, c->stream));
    if (v) HIPCHK(c, launch_transpose(v, c->mn->va, static_cast<int>(T), static_cast<int>(K * N), c->stream));
    HIPCHK(c, launch_mnmf_h(c->mn->tp, c->mn->va, p.v, p.F, p.T, p.N, c->mn->K, c->stream));
    HIPCHK(c, launch_fill_int(c->d_status, p.F, ST_OK, c->stream));
    HIPCHK(c, launch_fill_int(c->mn->vflag, 1, 0, c->stream));
    return FASTFCA_OK;
}

int fastfca_block_length(const fastfca_ctx *c, int b) {
    if (!c || b < 0 || b >= static_cast<int>(c->probs.size())) return FASTFCA_E_ARG;
    return c->probs[b].blocks ? c->probs[b].B : 0;
}

int fastfca_em_step(fastfca_ctx *c, int n_iter) {
    if (!c) return FASTFCA_E_ARG;
    if (n_iter < 1) return set_err(c, FASTFCA_E_ARG, "n_iter must be >= 1");
    if (n_iter > c->trace_cap) {
        int rc = upload_items(c, n_iter);
        if (rc != FASTFCA_OK) return rc;
    }
    c->last_n_iter = n_iter;
    // One class (a single mixture, or a batch of equal shapes) is one launch,
    // plus the tail split's few: launched directly, which leaves the stream
    // free a few microseconds sooner than a graph does. Batches of several
    // classes, the persistent queue and FastMNMF (three launches per
    // iteration) replay a graph captured once per n_iter.
    if (!c->mn && !c->persistent && c->classes.size() == 1) return record_em(c, n_iter);
    if (c->graph_exec && c->graph_n_iter == n_iter) {
        HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
        return FASTFCA_OK;
    }
    drop_graph(c);
    // capture the launch sequence once per n_iter, replay on later calls
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        int rc = record_em(c, n_iter);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        if (rc != FASTFCA_OK) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e2 == hipSuccess && g) {
            hipGraphExec_t ge = nullptr;
            if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess) {
                c->graph = g;
                c->graph_exec = ge;
                c->graph_n_iter = n_iter;
                HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
                return FASTFCA_OK;
            }
            hipGraphDestroy(g);
        }
        (void)hipGetLastError();
    } else {
        (void)hipGetLastError();
    }
    // capture unavailable (e.g. legacy default stream): launch directly
    return record_em(c, n_iter);
}

int fastfca_sync(fastfca_ctx *c) {
    if (!c) return FASTFCA_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_status(c);
}

int fastfca_loglik(fastfca_ctx *c, int b, double *ll_per_bin, double *ll_per_f) {
    if (!valid_problem(c, b)) return c ? set_err(c, FASTFCA_E_ARG, "bad mixture index %d", b) : FASTFCA_E_ARG;
    auto &p = c->probs[b];
    hipError_t e = launch_ldet(p.items, p.F, p.M, p.ldet, c->stream);
    if (e == hipSuccess) e = launch_loglik_terms(p.items, p.F, p.M, p.ldet, p.llf, c->stream);
    std::vector<double> llf(p.F);
    if (e == hipSuccess)
        e = hipMemcpyAsync(llf.data(), p.llf, sizeof(double) * p.F, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && ll_per_f)
        e = hipMemcpyAsync(ll_per_f, p.llf, sizeof(double) * p.F, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return set_err(c, FASTFCA_E_HIP, "loglik: %s", hipGetErrorString(e));
    int rc = check_status(c);
    if (rc != FASTFCA_OK) return rc;
    double s = 0.0;
    for (double v : llf) s += v;
    if (ll_per_bin) *ll_per_bin = s / p.F;
    if (!std::isfinite(s)) return set_err(c, FASTFCA_E_NONFINITE, "mixture %d: non-finite log-likelihood", b);
    return FASTFCA_OK;
}

int fastfca_ll_trace(fastfca_ctx *c, int b, double *trace, int max_n) {
    if (!valid_problem(c, b) || !trace || max_n < 0) return c ? set_err(c, FASTFCA_E_ARG, "bad arguments") : FASTFCA_E_ARG;
    if (c->last_n_iter == 0) return 0;
    auto &p = c->probs[b];
    const int n = std::min(max_n, c->last_n_iter);
    std::vector<double> buf(static_cast<size_t>(p.F) * c->trace_cap);
    HIPCHK(c, hipMemcpyAsync(buf.data(), c->d_trace + static_cast<size_t>(p.item0) * c->trace_cap,
                             sizeof(double) * buf.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int rc = check_status(c);
    if (rc != FASTFCA_OK) return rc;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int f = 0; f < p.F; ++f) s += buf[static_cast<size_t>(f) * c->trace_cap + i];
        trace[i] = s / p.F;
    }
    return n;
}

int fastfca_mwf(fastfca_ctx *c, int b, fastfca_c64 *y) {
    if (!valid_problem(c, b) || !y) return c ? set_err(c, FASTFCA_E_ARG, "bad arguments") : FASTFCA_E_ARG;
    auto &p = c->probs[b];
    HIPCHK(c, launch_mwf_bins(p.items, p.F, p.T * p.B, p.M, reinterpret_cast<float2 *>(y), c->stream));
    return FASTFCA_OK;
}

int fastfca_get_params(fastfca_ctx *c, int b, fastfca_c128 *P, float *lambda, float *v) {
    if (!valid_problem(c, b)) return c ? set_err(c, FASTFCA_E_ARG, "bad mixture index %d", b) : FASTFCA_E_ARG;
    auto &p = c->probs[b];
    const size_t F = p.F, T = p.T, M = p.M, N = p.N;
    if (P) HIPCHK(c, hipMemcpyAsync(P, p.P, sizeof(double2) * F * M * M, hipMemcpyDeviceToDevice, c->stream));
    if (lambda)
        HIPCHK(c, hipMemcpyAsync(lambda, p.lam, sizeof(float) * F * N * M, hipMemcpyDeviceToDevice, c->stream));
    if (v) HIPCHK(c, hipMemcpyAsync(v, p.v, sizeof(float) * F * T * N, hipMemcpyDeviceToDevice, c->stream));
    return FASTFCA_OK;
}

int fastfca_set_params(fastfca_ctx *c, int b, const fastfca_c128 *P, const float *lambda,
                       const float *v) {
    if (!valid_problem(c, b)) return c ? set_err(c, FASTFCA_E_ARG, "bad mixture index %d", b) : FASTFCA_E_ARG;
    auto &p = c->probs[b];
    const size_t F = p.F, T = p.T, M = p.M, N = p.N;
    // one launch for the three copies and the status reset
    HIPCHK(c, launch_set_params(p.P, reinterpret_cast<const double2 *>(P), F * M * M, p.lam, lambda, F * N * M,
                                p.v, v, F * T * N, c->d_status + p.item0, p.F, c->stream));
    return FASTFCA_OK;
}

int fastfca_shape(const fastfca_ctx *c, int b, int *F, int *T, int *M, int *N) {
    if (!c || b < 0 || b >= static_cast<int>(c->probs.size())) return FASTFCA_E_ARG;
    const auto &p = c->probs[b];
    if (F) *F = p.F;
    if (T) *T = p.T;
    if (M) *M = p.M;
    if (N) *N = p.N;
    return FASTFCA_OK;
}

int fastfca_num_problems(const fastfca_ctx *c) { return c ? static_cast<int>(c->probs.size()) : FASTFCA_E_ARG; }

int fastfca_set_config(fastfca_ctx *c, int threads, int bins_per_thread) {
    if (!c) return FASTFCA_E_ARG;
    if (c->mn) return set_err(c, FASTFCA_E_STATE, "FastMNMF contexts use a fixed launch shape");
    if (threads == 0 && bins_per_thread == 0) {
        for (auto &cc : c->classes) pick_class(cc);
        drop_graph(c);
        return FASTFCA_OK;
    }
    if (threads < 64 || (threads & 63) || threads * bins_per_thread > kWideMaxT ||
        (bins_per_thread != 2 && bins_per_thread != 4 && bins_per_thread != 8 &&
         bins_per_thread != 16))
        return set_err(c, FASTFCA_E_ARG, "invalid config threads=%d bins_per_thread=%d", threads,
                       bins_per_thread);
    for (auto &cc : c->classes) {
        if (threads * bins_per_thread < cc.Tmax)
            return set_err(c, FASTFCA_E_ARG, "threads*bins_per_thread=%d < T=%d",
                           threads * bins_per_thread, cc.Tmax);
        if (!cc.wide && !em_supported(cc.M, cc.N, bins_per_thread, cc.cov))
            return set_err(c, FASTFCA_E_ARG, "no kernel with %d bins per thread for M=%d N=%d",
                           bins_per_thread, cc.M, cc.N);
        if (!cc.wide && threads * bins_per_thread > kResidentBins)
            return set_err(c, FASTFCA_E_ARG, "threads*bins_per_thread=%d > 2048 for M=%d N=%d",
                           threads * bins_per_thread, cc.M, cc.N);
        if (cc.wide && (threads * bins_per_thread > kWideMaxT || threads > wide_max_threads(bins_per_thread) ||
                        !em_wide_supported(cc.M, cc.N, bins_per_thread)))
            return set_err(c, FASTFCA_E_ARG, "M=%d N=%d T=%d: the wide kernels take 4 or 8 bins per "
                           "thread, at most 512 threads and at most 4096 bins", cc.M, cc.N, cc.Tmax);
    }
    if (c->persistent) {
        c->p_threads = threads;
        c->p_bpt = bins_per_thread;
    } else {
        for (auto &cc : c->classes) {
            cc.threads = threads;
            cc.bpt = bins_per_thread;
        }
    }
    drop_graph(c);
    return FASTFCA_OK;
}

int fastfca_set_ll_alarm(fastfca_ctx *c, double tol) {
    if (!c) return FASTFCA_E_ARG;
    if (tol != tol) return set_err(c, FASTFCA_E_ARG, "ll alarm tolerance is NaN");
    if (tol != c->ll_alarm) drop_graph(c);
    c->ll_alarm = tol;
    return FASTFCA_OK;
}

int fastfca_set_tail_split(fastfca_ctx *c, int blocks) {
    if (!c) return FASTFCA_E_ARG;
    if (blocks < -1 || blocks > 1024)
        return set_err(c, FASTFCA_E_ARG, "tail split %d: -1 (automatic), 0 (off) or 1..1024 blocks", blocks);
    if (blocks != c->tail_split) drop_graph(c);
    c->tail_split = blocks;
    return FASTFCA_OK;
}

int fastfca_set_algorithm(fastfca_ctx *c, int algo) {
    if (!c) return FASTFCA_E_ARG;
    if (algo != FASTFCA_ALGO_EM && algo != FASTFCA_ALGO_MM)
        return set_err(c, FASTFCA_E_ARG, "unknown algorithm %d", algo);
    if (c->mn) return set_err(c, FASTFCA_E_UNSUPPORTED, "FastMNMF updates Lambda, T and V by MM only");
    c->algo = algo == FASTFCA_ALGO_MM ? kAlgoMM : kAlgoEM;
    drop_graph(c);
    return FASTFCA_OK;
}

int fastfca_set_schedule(fastfca_ctx *c, int schedule) {
    if (!c) return FASTFCA_E_ARG;
    if (schedule != FASTFCA_SCHEDULE_CLASSES && schedule != FASTFCA_SCHEDULE_PERSISTENT)
        return set_err(c, FASTFCA_E_ARG, "unknown schedule %d", schedule);
    if (c->mn) return set_err(c, FASTFCA_E_STATE, "FastMNMF contexts use a fixed schedule");
    const bool want = schedule == FASTFCA_SCHEDULE_PERSISTENT;
    if (want == c->persistent) return FASTFCA_OK;
    if (want) {
        if (c->probs.size() < 2 || !c->p_threads)
            return set_err(c, FASTFCA_E_UNSUPPORTED, "the persistent schedule needs a batch of supported classes");
    }
    int rc = fastfca_sync(c);
    if (rc != FASTFCA_OK) return rc;
    c->persistent = want;
    drop_graph(c);
    return upload_items(c, c->trace_cap);
}

int fastfca_get_config(const fastfca_ctx *c, int b, int *threads, int *bins_per_thread) {
    if (!c || b < 0 || b >= static_cast<int>(c->probs.size())) return FASTFCA_E_ARG;
    if (c->persistent) {
        if (threads) *threads = c->p_threads;
        if (bins_per_thread) *bins_per_thread = c->p_bpt;
        return FASTFCA_OK;
    }
    const auto &cc = c->classes[c->h_items[c->probs[b].item0].cls];
    if (threads) *threads = cc.threads;
    if (bins_per_thread) *bins_per_thread = cc.bpt;
    return FASTFCA_OK;
}

int fastfca_autotune(fastfca_ctx *c, int n_iter, const char *cache_path) {
    if (!c || n_iter < 1) return c ? set_err(c, FASTFCA_E_ARG, "n_iter must be >= 1") : FASTFCA_E_ARG;
    if (c->mn) return set_err(c, FASTFCA_E_STATE, "FastMNMF contexts use a fixed launch shape");
    int rc = fastfca_sync(c);
    if (rc != FASTFCA_OK) return rc;
    if (n_iter > c->trace_cap && (rc = upload_items(c, n_iter)) != FASTFCA_OK) return rc;
    // snapshot the state: trials run on the live buffers and are undone
    struct Snap {
        float *v, *lam;
        double2 *P;
    };
    std::vector<Snap> snaps(c->probs.size(), Snap{nullptr, nullptr, nullptr});
    auto free_snaps = [&]() {
        for (auto &s : snaps) {
            hipFree(s.v);
            hipFree(s.lam);
            hipFree(s.P);
        }
    };
    for (size_t b = 0; b < c->probs.size() && rc == FASTFCA_OK; ++b) {
        auto &p = c->probs[b];
        const size_t F = p.F, T = p.T, M = p.M, N = p.N;
        if ((rc = dalloc(c, &snaps[b].v, F * T * N)) != FASTFCA_OK) break;
        if ((rc = dalloc(c, &snaps[b].lam, F * N * M)) != FASTFCA_OK) break;
        if ((rc = dalloc(c, &snaps[b].P, F * M * M)) != FASTFCA_OK) break;
        hipMemcpyAsync(snaps[b].v, p.v, sizeof(float) * F * T * N, hipMemcpyDeviceToDevice, c->stream);
        hipMemcpyAsync(snaps[b].lam, p.lam, sizeof(float) * F * N * M, hipMemcpyDeviceToDevice, c->stream);
        hipMemcpyAsync(snaps[b].P, p.P, sizeof(double2) * F * M * M, hipMemcpyDeviceToDevice, c->stream);
    }
    if (rc != FASTFCA_OK) {
        free_snaps();
        return rc;
    }
    auto restore = [&]() {
        for (size_t b = 0; b < c->probs.size(); ++b) {
            auto &p = c->probs[b];
            const size_t F = p.F, T = p.T, M = p.M, N = p.N;
            hipMemcpyAsync(p.v, snaps[b].v, sizeof(float) * F * T * N, hipMemcpyDeviceToDevice, c->stream);
            hipMemcpyAsync(p.lam, snaps[b].lam, sizeof(float) * F * N * M, hipMemcpyDeviceToDevice, c->stream);
            hipMemcpyAsync(p.P, snaps[b].P, sizeof(double2) * F * M * M, hipMemcpyDeviceToDevice, c->stream);
        }
        launch_fill_int(c->d_status, static_cast<int>(c->h_items.size()), ST_OK, c->stream);
    };
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    auto time_once = [&](float &ms) -> int {
        restore();
        HIPCHK(c, hipEventRecord(e0, c->stream));
        int r = record_em(c, n_iter);
        if (r != FASTFCA_OK) return r;
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        return FASTFCA_OK;
    };
    auto best_of = [&](float &best) -> int {
        best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            float ms = 0.f;
            int r = time_once(ms);
            if (r != FASTFCA_OK) return r;
            best = std::min(best, ms);
        }
        return FASTFCA_OK;
    };
    FILE *cache = cache_path ? fopen(cache_path, "a") : nullptr;
    auto bucket = [](int T) {
        int b = 64;
        while (b < T) b <<= 1;
        return b;
    };
    if (c->probs.size() > 1) {
        // batch: the class schedule at its default shapes against the
        // persistent queue at each admissible shape and grid
        int Tmax = 0;
        for (auto &cc : c->classes) Tmax = std::max(Tmax, cc.Tmax);
        float cls_ms = 1e30f, best = 1e30f;
        c->persistent = false;
        rc = upload_items(c, c->trace_cap);
        if (rc == FASTFCA_OK) rc = best_of(cls_ms);
        int bt = c->p_threads, bb = c->p_bpt, bg = c->p_grid;
        if (rc == FASTFCA_OK && c->p_threads) {
            int ncu = 256;
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
            c->persistent = true;
            rc = upload_items(c, c->trace_cap);
            for (int bpt : {4, 8}) {
                const int th = threads_for(Tmax, bpt);
                if (!th || rc != FASTFCA_OK) continue;
                for (int per_cu : {1, 2, 4}) {
                    c->p_threads = th;
                    c->p_bpt = bpt;
                    c->p_grid = ncu * per_cu;
                    float ms;
                    rc = best_of(ms);
                    if (rc != FASTFCA_OK) break;
                    if (ms < best) {
                        best = ms;
                        bt = th;
                        bb = bpt;
                        bg = c->p_grid;
                    }
                }
            }
            c->p_threads = bt;
            c->p_bpt = bb;
            c->p_grid = bg;
        }
        if (rc == FASTFCA_OK) {
            c->persistent = best < cls_ms;
            rc = upload_items(c, c->trace_cap);
        }
        if (cache && rc == FASTFCA_OK)
            fprintf(cache,
                    "{\"arch\": \"%s\", \"kind\": \"batch\", \"items\": %zu, \"Tbucket\": %d, "
                    "\"class_launches_ms\": %.6f, \"persistent_ms\": %.6f, \"threads\": %d, "
                    "\"bins_per_thread\": %d, \"grid\": %d, \"persistent\": %d}\n",
                    c->arch, c->h_items.size(), bucket(Tmax), cls_ms, best, bt, bb, bg, c->persistent ? 1 : 0);
    } else {
        for (auto &cc : c->classes) {
            int bt = cc.threads, bb = cc.bpt;
            float best = 1e30f;
            for (int bpt : {2, 4, 8, 16}) {
                const int th = threads_for(cc.Tmax, bpt, cc.wide ? kWideMaxT : kResidentBins);
                if (!th || (cc.wide && th > wide_max_threads(bpt))) continue;
                if (cc.wide ? !em_wide_supported(cc.M, cc.N, bpt) : !em_supported(cc.M, cc.N, bpt, cc.cov))
                    continue;
                cc.threads = th;
                cc.bpt = bpt;
                float ms;
                rc = best_of(ms);
                if (rc != FASTFCA_OK) break;
                if (ms < best) {
                    best = ms;
                    bt = th;
                    bb = bpt;
                }
            }
            cc.threads = bt;
            cc.bpt = bb;
            if (rc != FASTFCA_OK) break;
            if (cache)
                fprintf(cache,
                        "{\"arch\": \"%s\", \"kind\": \"class\", \"M\": %d, \"N\": %d, \"Tbucket\": %d, "
                        "\"threads\": %d, \"bins_per_thread\": %d, \"ms\": %.6f}\n",
                        c->arch, cc.M, cc.N, bucket(cc.Tmax), bt, bb, best);
        }
    }
    if (cache) fclose(cache);
    restore();
    hipError_t e = hipStreamSynchronize(c->stream);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    free_snaps();
    drop_graph(c);
    if (rc == FASTFCA_OK && e != hipSuccess)
        rc = set_err(c, FASTFCA_E_HIP, "autotune: %s", hipGetErrorString(e));
    return rc;
}

int fastfca_synth_mixture(fastfca_c64 *x, int F, int T, int M, int N, int rank, float diffuse,
                          uint64_t seed, void *hip_stream) {
    if (!x || F < 1 || T < 1 || M < 1 || M > 8 || N < 1 || rank < 1 || !(diffuse >= 0.0f))
        return set_err(nullptr, FASTFCA_E_ARG, "synth: invalid arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    float *W = nullptr;
    float2 *C = nullptr;
    hipError_t e = hipMalloc(&W, sizeof(float) * static_cast<size_t>(N) * F * rank);
    if (e == hipSuccess) e = hipMalloc(&C, sizeof(float2) * static_cast<size_t>(N) * F * M * M);
    if (e == hipSuccess)
        e = launch_synth(reinterpret_cast<float2 *>(x), F, T, M, N, rank, diffuse, seed, W, C, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(W);
    hipFree(C);
    if (e != hipSuccess) return set_err(nullptr, FASTFCA_E_HIP, "synth: %s", hipGetErrorString(e));
    return FASTFCA_OK;
}

int fastfca_fit_noalloc(const fastfca_c64 *x, int F, int T, int M, int N, fastfca_c128 *P, float *lambda,
                        float *v, int n_iter, int *status, double *ll_trace, void *hip_stream) {
    if (!x || !P || !lambda || !v || !status)
        return noalloc_err(FASTFCA_E_ARG, "fit_noalloc: x, P, lambda, v and status are required");
    if (F < 1 || T < 1 || M < 2 || N < 2 || T < M || n_iter < 1)
        return noalloc_err(FASTFCA_E_ARG, "fit_noalloc: invalid F=%d T=%d M=%d N=%d n_iter=%d", F, T, M, N, n_iter);
    ClassCfg cc{M, N, T};
    if (M > FASTFCA_MAX_M || N > FASTFCA_MAX_N || T > FASTFCA_MAX_T || !pick_class(cc))
        return noalloc_err(FASTFCA_E_UNSUPPORTED, "fit_noalloc: no compiled kernel for M=%d N=%d T=%d", M, N, T);
    const size_t items_b = align256(sizeof(WorkItem) * static_cast<size_t>(F));
    const size_t ldet_b = align256(sizeof(double) * static_cast<size_t>(F));
    const size_t trace_b = ll_trace ? 0 : align256(sizeof(double) * static_cast<size_t>(F) * n_iter);
    if (items_b + ldet_b + trace_b > FASTFCA_NOALLOC_SCRATCH_BYTES)
        return noalloc_err(FASTFCA_E_ARG,
                           "fit_noalloc: F=%d n_iter=%d needs %zu bytes of scratch, more than the %u available%s", F,
                           n_iter, items_b + ldet_b + trace_b, FASTFCA_NOALLOC_SCRATCH_BYTES,
                           ll_trace ? "" : " (pass ll_trace to keep the trace out of it)");
    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc != FASTFCA_OK) return rc;
    unsigned char *sp = static_cast<unsigned char *>(base);
    WorkItem *items = reinterpret_cast<WorkItem *>(sp);
    double *ldet = reinterpret_cast<double *>(sp + items_b);
    double *trace = ll_trace ? ll_trace : reinterpret_cast<double *>(sp + items_b + ldet_b);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(noalloc_items_kernel, dim3((F + 255) / 256), dim3(256), 0, s, items,
                       reinterpret_cast<const float2 *>(x), reinterpret_cast<double2 *>(P), lambda, v, trace, n_iter,
                       ldet, status, F, T, M, N);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        const EmLaunch a{items, F, n_iter, nullptr, kAlgoEM, kDefaultLLAlarm};
        e = cc.wide ? launch_em_wide(M, N, cc.bpt, cc.threads, a, F, s) : launch_em(M, N, cc.bpt, cc.threads, a, F, s);
    }
    if (e != hipSuccess) return noalloc_err(FASTFCA_E_HIP, "fit_noalloc: launch failed: %s", hipGetErrorString(e));
    return FASTFCA_OK;
}

const char *fastfca_last_error(const fastfca_ctx *c) {
    if (c) return c->err.c_str();
    return g_noalloc_error_newer ? g_noalloc_error : g_init_error.c_str();
}

void fastfca_destroy(fastfca_ctx *c) {
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    drop_graph(c);
    for (int q = 0; q < fastfca_ctx::kSide; ++q) {
        if (c->side[q]) {
            hipStreamSynchronize(c->side[q]);
            hipStreamDestroy(c->side[q]);
        }
        if (c->join[q]) hipEventDestroy(c->join[q]);
    }
    if (c->fork) hipEventDestroy(c->fork);
    for (auto &p : c->probs) free_problem(p);
    if (c->mn) {
        hipFree(c->mn->tp);
        hipFree(c->mn->va);
        hipFree(c->mn->G);
        hipFree(c->mn->E);
        hipFree(c->mn->part);
        hipFree(c->mn->vflag);
        delete c->mn;
    }
    hipFree(c->ws.feat.p);
    hipFree(c->ws.lv.p);
    hipFree(c->ws.part.p);
    hipFree(c->ws.pooled.p);
    hipFree(c->ws.ll.p);
    hipFree(c->ws.P_old.p);
    hipFree(c->ws.lam_old.p);
    hipFree(c->ws.v_old.p);
    hipFree(c->ws.ll_old.p);
    hipFree(c->ws.ll_new.p);
    hipFree(c->ws.taken.p);
    hipFree(c->d_items);
    hipFree(c->d_status);
    hipFree(c->d_trace);
    hipFree(c->d_queue);
    delete c;
}

}  // extern "C"

namespace {

// Argument checks shared by the two warm-start entry points.
int ws_check(fastfca_ctx *c, int b, const fastfca_net *net) {
    if (!valid_problem(c, b)) return c ? set_err(c, FASTFCA_E_ARG, "bad mixture index %d", b) : FASTFCA_E_ARG;
    auto &p = c->probs[b];
    if (p.blocks || c->mn) return set_err(c, FASTFCA_E_STATE, "warm start: frame-model contexts only");
    if (p.M > 4) return set_err(c, FASTFCA_E_ARG, "warm start: M = %d > 4", p.M);
    if (net) {
        if (net->M != p.M || net->N != p.N)
            return set_err(c, FASTFCA_E_ARG, "warm start: network for M=%d N=%d, mixture %d has M=%d N=%d", net->M,
                           net->N, b, p.M, p.N);
        if (net->C < 16 || net->C > 64 || net->C % 16 || net->L < 0 || net->L > 8 || net->N > 8 || !net->Wb ||
            !net->b || !net->Wv || !net->bv || !net->Wl || !net->bl || net->ldv < net->C ||
            (net->Kp0 != 16 && net->Kp0 != 32) || net->Kp0 < 5 * net->M)
            return set_err(c, FASTFCA_E_ARG, "warm start: unsupported network (C=%d L=%d Kp0=%d)", net->C, net->L,
                           net->Kp0);
        for (int l = 0; l <= net->L; ++l)
            if (!net->Wb[l] || !net->b[l]) return set_err(c, FASTFCA_E_ARG, "warm start: layer %d missing", l);
    }
    return FASTFCA_OK;
}

// The new start of mixture b written over its state (features, and the
// network's outputs or the whitening-only start), with the workspace it needs.
int ws_new_start(fastfca_ctx *c, int b, const fastfca_net *net) {
    auto &p = c->probs[b];
    const size_t F = p.F, T = p.T, M = p.M, N = p.N;
    auto &w = c->ws;
    int rc = FASTFCA_OK;
    if ((rc = ws_reserve(c, w.feat, F * M * T)) != FASTFCA_OK) return rc;
    if (net && ((rc = ws_reserve(c, w.lv, F * N * T)) != FASTFCA_OK ||
                (rc = ws_reserve(c, w.part, F * ((T + 63) / 64) * net->C)) != FASTFCA_OK ||
                (rc = ws_reserve(c, w.pooled, F * net->C)) != FASTFCA_OK || (rc = ws_reserve(c, w.ll, F * N * M)) != FASTFCA_OK))
        return rc;
    hipStream_t s = c->stream;
    // whitening P0 = C_f^{-1/2}, written as the new P, and the features
    HIPCHK(c, net_features(p.x, p.F, p.T, p.M, 1e-8f, p.P, w.feat.p, s));
    if (net) {
        HIPCHK(c, net_forward_fused(w.feat.p, p.F, p.M, p.T, net->C, net->L, p.N, net->Wb, net->b, net->Kp0, net->Wv,
                                    net->ldv, net->bv, w.lv.p, w.part.p, w.pooled.p, s));
        HIPCHK(c, net_linear_fwd(w.pooled.p, p.F, net->C, net->Wl, net->bl, p.N * p.M, w.ll.p, s));
        HIPCHK(c, net_apply_outputs(w.lv.p, w.ll.p, p.F, p.T, p.M, p.N, p.v, p.lam, s));
    } else {
        HIPCHK(c, launch_ws_whitened(p.x, p.P, p.lam, p.v, p.F, p.T, p.M, p.N, s));
    }
    return FASTFCA_OK;
}

}  // namespace

extern "C" {

int fastfca_warmstart(fastfca_ctx *c, int b, const fastfca_net *net, int *n_taken) {
    int rc = ws_check(c, b, net);
    if (rc != FASTFCA_OK) return rc;
    auto &p = c->probs[b];
    const size_t F = p.F, T = p.T, M = p.M, N = p.N;
    auto &w = c->ws;
    if ((rc = ws_reserve(c, w.P_old, F * M * M)) != FASTFCA_OK || (rc = ws_reserve(c, w.lam_old, F * N * M)) != FASTFCA_OK ||
        (rc = ws_reserve(c, w.v_old, F * T * N)) != FASTFCA_OK || (rc = ws_reserve(c, w.ll_old, F)) != FASTFCA_OK ||
        (rc = ws_reserve(c, w.ll_new, F)) != FASTFCA_OK || (rc = ws_reserve(c, w.taken, 1)) != FASTFCA_OK)
        return rc;
    hipStream_t s = c->stream;
    // the start being replaced and its likelihood per frequency
    HIPCHK(c, hipMemcpyAsync(w.P_old.p, p.P, sizeof(double2) * F * M * M, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(w.lam_old.p, p.lam, sizeof(float) * F * N * M, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(w.v_old.p, p.v, sizeof(float) * F * T * N, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, launch_ldet(p.items, p.F, p.M, p.ldet, s));
    HIPCHK(c, launch_loglik_terms(p.items, p.F, p.M, p.ldet, w.ll_old.p, s));
    if ((rc = ws_new_start(c, b, net)) != FASTFCA_OK) return rc;
    // judge: the new start's likelihood against the old one's, per frequency
    HIPCHK(c, launch_ldet(p.items, p.F, p.M, p.ldet, s));
    HIPCHK(c, launch_loglik_terms(p.items, p.F, p.M, p.ldet, w.ll_new.p, s));
    HIPCHK(c, launch_fill_int(w.taken.p, 1, 0, s));
    HIPCHK(c, launch_ws_select(w.ll_old.p, w.ll_new.p, p.P, p.lam, p.v, w.P_old.p, w.lam_old.p, w.v_old.p, p.F, p.T, p.M,
                               p.N, w.taken.p, s));
    // the likelihood kernels record a singular P of a rejected start
    HIPCHK(c, launch_fill_int(c->d_status + p.item0, p.F, ST_OK, s));
    if (n_taken) {
        int h = 0;
        HIPCHK(c, hipMemcpyAsync(&h, w.taken.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        *n_taken = h;
    }
    return FASTFCA_OK;
}

int fastfca_warmstart_race(fastfca_ctx *c, int b, const fastfca_net *net, int race_iters, int *n_taken) {
    int rc = ws_check(c, b, net);
    if (rc != FASTFCA_OK) return rc;
    if (race_iters < 1) return set_err(c, FASTFCA_E_ARG, "warm start race: race_iters = %d < 1", race_iters);
    auto &p = c->probs[b];
    const size_t F = p.F, T = p.T, M = p.M, N = p.N, K = race_iters;
    auto &w = c->ws;
    if ((rc = ws_reserve(c, w.P_old, F * M * M)) != FASTFCA_OK || (rc = ws_reserve(c, w.lam_old, F * N * M)) != FASTFCA_OK ||
        (rc = ws_reserve(c, w.v_old, F * T * N)) != FASTFCA_OK || (rc = ws_reserve(c, w.ll_old, F)) != FASTFCA_OK ||
        (rc = ws_reserve(c, w.ll_new, F)) != FASTFCA_OK || (rc = ws_reserve(c, w.taken, 1)) != FASTFCA_OK ||
        (rc = ws_reserve(c, w.race_trace, 2 * F * K)) != FASTFCA_OK || (rc = ws_reserve(c, w.race_ldet, F)) != FASTFCA_OK ||
        (rc = ws_reserve(c, w.race_status, F)) != FASTFCA_OK || (rc = ws_reserve(c, w.race_items, 2 * F)) != FASTFCA_OK)
        return rc;
    hipStream_t s = c->stream;
    int *st_b = c->d_status + p.item0;
    // start A, the current state, set aside; start B written over the state
    HIPCHK(c, hipMemcpyAsync(w.P_old.p, p.P, sizeof(double2) * F * M * M, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(w.lam_old.p, p.lam, sizeof(float) * F * N * M, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(w.v_old.p, p.v, sizeof(float) * F * T * N, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, launch_fill_int(w.race_status.p, p.F, ST_OK, s));
    HIPCHK(c, launch_fill_int(st_b, p.F, ST_OK, s));
    if ((rc = ws_new_start(c, b, net)) != FASTFCA_OK) return rc;
    // the work table of the race: B on the mixture's own state, A on the
    // copy; each frequency's trace row holds K entries
    std::vector<WorkItem> tab(2 * F);
    for (size_t f = 0; f < F; ++f) {
        WorkItem it = c->h_items[p.item0 + f];
        it.status = st_b + f;
        it.ll_trace = w.race_trace.p + f * K;
        tab[f] = it;
        it.P = w.P_old.p + f * M * M;
        it.lam = w.lam_old.p + f * N * M;
        it.v = w.v_old.p + f * T * N;
        it.ldet = w.race_ldet.p + f;
        it.status = w.race_status.p + f;
        it.ll_trace = w.race_trace.p + (F + f) * K;
        tab[F + f] = it;
    }
    const bool same = w.race_host.size() == tab.size() &&
                      std::memcmp(w.race_host.data(), tab.data(), sizeof(WorkItem) * tab.size()) == 0;
    if (!same) {
        w.race_host = tab;
        HIPCHK(c, hipMemcpyAsync(w.race_items.p, w.race_host.data(), sizeof(WorkItem) * tab.size(),
                                 hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));  // the host table may change on the next call
    }
    // both starts, race_iters iterations of the context's algorithm, in one launch
    const auto &cc = c->classes[c->h_items[p.item0].cls];
    EmLaunch a{w.race_items.p, static_cast<int>(2 * F), race_iters, nullptr, c->algo, c->ll_alarm, 0, 0};
    HIPCHK(c, launch_class(cc, a, static_cast<int>(2 * F), s));
    // keep per frequency the start with the higher likelihood after the race
    HIPCHK(c, launch_race_ll(w.race_trace.p, race_iters, st_b, w.race_status.p, w.ll_new.p, w.ll_old.p, p.F, s));
    HIPCHK(c, launch_fill_int(w.taken.p, 1, 0, s));
    HIPCHK(c, launch_ws_select(w.ll_old.p, w.ll_new.p, p.P, p.lam, p.v, w.P_old.p, w.lam_old.p, w.v_old.p, p.F, p.T, p.M,
                               p.N, w.taken.p, s, st_b, w.race_status.p, p.ldet, w.race_ldet.p));
    if (n_taken) {
        int h = 0;
        HIPCHK(c, hipMemcpyAsync(&h, w.taken.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        *n_taken = h;
    }
    return FASTFCA_OK;
}

}  // extern "C"
