// Internal declarations shared by the kernels and the host runtime of the
// FastFCA library. Not part of the public ABI (include/fastfca.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffca {

// One unit of GPU work: one frequency of one mixture. Every array pointer
// addresses that frequency's slice in the library's own buffers.
struct WorkItem {
    const float2 *x;   // [Tx][M] mixture STFT frames
    const float *z;    // [T][M*M] block covariances of the piecewise stationary
                       // model (diagonal, then re/im of the upper triangle), or
                       // nullptr when every bin is one frame (z_t = x_t x_t^H)
    float *v;          // [T][N]  source powers h_{tn} (one per bin or block)
    float *lam;        // [N][M]  diag(Lambda_n)
    double2 *P;        // [M][M]  decorrelation matrix, double precision master
    double *ll_trace;  // [trace_stride] LL per bin after each iteration
    double *ldet;      // ln|det P|^2 after the last IP sweep
    int *status;       // 0 = ok, else FASTFCA_E_* recorded by the kernel
    int T, M, N;       // T: bins the iteration runs over (frames, or blocks)
    int B;             // frames per bin: 1, or the block length
    int Tx;            // frames in x (T * B)
    int cls;           // kernel class index (M, N) used by the persistent launch
};

// Status codes written by kernels (mirror the public ABI values).
enum : int { ST_OK = 0, ST_SINGULAR = -4, ST_NONFINITE = -5, ST_DECREASE = -8 };

// Largest T handled by the resident IP+EM kernels: a workgroup holds at most
// kResidentBins bins (threads * bins-per-thread), with threads <= 2048 / BPT.
constexpr int kResidentBins = 2048;

// Relative pivot threshold of the double precision IP solve.
constexpr double kPivotTol = 1e-12;

// Update of L and H inside an iteration: Algorithm 1 (EM, sequential over
// sources) or Algorithm 2 (MM, all sources at once).
enum : int { kAlgoEM = 0, kAlgoMM = 1 };

struct EmLaunch {
    const WorkItem *items;  // items handled by this launch
    int n_items;
    int n_iter;
    int *queue;             // persistent launch: next-item counter (nullptr otherwise)
    int algo;               // kAlgoEM or kAlgoMM
    double ll_alarm;        // a frequency whose LL per bin falls by more than this between two
                            // iterations of a call is stopped with ST_DECREASE (+inf: never)
    int trace_off;          // first trace entry this launch writes (a launch that continues a
                            // call's iterations writes after the entries already written)
    int prio;               // 1: a tail launch, run by the kernels' tail instance (highest wave
                            // issue priority on its SIMD)
};

// Launch one EM kernel (Algorithm 1 for n_iter iterations) over `n_items`
// work items that share (M, N). bpt: bins per thread held in registers.
// cov: the items carry block covariances (piecewise stationary model).
hipError_t launch_em(int M, int N, int bpt, int threads, const EmLaunch &a, int grid,
                     hipStream_t s, bool cov = false);
bool em_supported(int M, int N, int bpt, bool cov = false);
// Workgroups of the resident kernel (M, N, bpt) with `threads` threads that
// one CU holds at once (0 if the kernel does not exist).
int em_blocks_per_cu(int M, int N, int bpt, int threads, bool cov = false);
using EmFn = void (*)(EmLaunch);
EmFn em_cov_lookup(int M, int N, int bpt, bool prio = false);
// A tail instance (highest wave priority) exists for this shape.
bool em_tail_supported(int M, int N, int bpt, bool cov = false);

// Wide family (M <= 8, N <= 12, T <= kWideBins = 4096): x is re-read from
// global memory each iteration; see em_wide.hpp. One lookup per M, defined in
// the per-M translation units of em_wide_kernel.hip.
template <int M>
void (*wide_lookup(int N, int bpt, bool prio, bool mm))(EmLaunch);
hipError_t launch_em_wide(int M, int N, int bpt, int threads, const EmLaunch &a, int grid,
                          hipStream_t s);
bool em_wide_supported(int M, int N, int bpt);
int em_wide_blocks_per_cu(int M, int N, int bpt, int threads);
bool em_wide_tail_supported(int M, int N, int bpt);
constexpr int kWideMaxT = 4096;
constexpr int kWideMaxThreads = 512;  // workgroup size limit of the wide kernels
// Workgroup size limit of a wide kernel with bpt bins per thread.
constexpr int wide_max_threads(int bpt) { return kWideMaxT / bpt < kWideMaxThreads ? kWideMaxT / bpt : kWideMaxThreads; }

// Persistent launch over a mixed list of work items (any supported (M, N) in
// the batch class table), pulling items from a device counter.
hipError_t launch_em_persistent(const EmLaunch &a, int threads, int bpt, int grid,
                                hipStream_t s);
bool persistent_supported(int M, int N);

// Double precision log-likelihood per frequency of one mixture.
hipError_t launch_loglik(const WorkItem *items, int n_items, int M, double *ll_f,
                         hipStream_t s);

// Multichannel Wiener filter of one mixture: y [N][F][T][M].
hipError_t launch_mwf(const WorkItem *items, int F, int T, int M, int N, float2 *y,
                      hipStream_t s);

// Initialization helpers.
hipError_t launch_check_finite_x(const float2 *x, size_t n, int *flag, hipStream_t s);
hipError_t launch_check_positive(const float *a, size_t n, int *flag, hipStream_t s);
hipError_t launch_identity_P(double2 *P, int F, int M, hipStream_t s);
// v from the frame power |x_t|^2 or, when z is given, from the block power tr(Xhat_j).
hipError_t launch_seeded_init(const float2 *x, const float *z, float *lam, float *v, int F, int T,
                              int M, int N, uint64_t seed, bool do_lam, bool do_v, hipStream_t s);
// Block covariances z [F][J][M*M] of x [F][J*B][M] (Sec. VI).
hipError_t launch_block_cov(const float2 *x, float *z, int F, int J, int B, int M, hipStream_t s);
hipError_t launch_fill_int(int *p, int n, int value, hipStream_t s);
// Copy P [nP], lambda [nl] and v [nv] (a NULL source skips that array) and
// set status[0..F) to ST_OK, in one launch.
hipError_t launch_set_params(double2 *P, const double2 *Ps, size_t nP, float *lam, const float *ls, size_t nl,
                             float *v, const float *vs, size_t nv, int *status, int F, hipStream_t s);

}  // namespace ffca
