// Kernels and dispatch of the IP+EM iteration; the per-item body is em_item.hpp.
#include "em_item.hpp"

namespace ffca {

// Register budget: a launch with BPT bins per thread uses at most 2048 / BPT
// threads (kMaxThreadsFor), which lets the compiler give each lane up to
// 128 (BPT 2), 256 (BPT 4) or 512 (BPT 8) VGPRs.
// M = 3 at eight bins per thread with up to five sources is held to 256
// VGPRs (two waves per SIMD); at N = 5 that costs some spills and still runs
// 26 % faster than one wave per SIMD at 275 VGPRs (513 frequencies,
// T = 2000). More sources would spill too much.
// PRIO: the instance for the tail launches of the tail split, whose waves take
// the highest issue priority on their SIMD so that the few frequencies they
// run keep pace next to a full grid. A separate instance, because the
// priority instruction in the common kernel changes its register allocation
// (twice the spills at M = 3, N = 5, eight bins per thread).
template <int M, int N, int BPT, bool PRIO>
__global__ void __launch_bounds__(kResidentBins / BPT)
    __attribute__((amdgpu_waves_per_eu(M == 3 && BPT == 8 && N <= 5 ? 2 : 1))) em_kernel(EmLaunch a) {
    __shared__ EmSmem<M * M * M, 2 * N * M, wave_slots(BPT)> sm;
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
    const WorkItem &it = a.items[blockIdx.x];
    if (*it.status != ST_OK) return;  // frozen after an earlier failure
    em_item<M, N, BPT, false>(it, a.n_iter, a.algo, a.ll_alarm, a.trace_off, sm);
}

// ------------------------------------------------------------------ dispatch

template <int M, int N>
struct BptTable {
    // tail instances (prio) exist for four and eight bins per thread
    static EmFn get(int bpt, bool prio) {
        switch (bpt) {
            case 2: return prio ? nullptr : em_kernel<M, N, 2, false>;
            case 4: return prio ? em_kernel<M, N, 4, true> : em_kernel<M, N, 4, false>;
            case 8: return prio ? em_kernel<M, N, 8, true> : em_kernel<M, N, 8, false>;
            case 16: return prio ? nullptr : em_kernel<M, N, 16, false>;
            default: return nullptr;
        }
    }
};

#define FFCA_N_CASES(M)                      \
    switch (N) {                             \
        case 2: return BptTable<M, 2>::get(bpt, prio); \
        case 3: return BptTable<M, 3>::get(bpt, prio); \
        case 4: return BptTable<M, 4>::get(bpt, prio); \
        case 5: return BptTable<M, 5>::get(bpt, prio); \
        case 6: return BptTable<M, 6>::get(bpt, prio); \
        case 7: return BptTable<M, 7>::get(bpt, prio); \
        case 8: return BptTable<M, 8>::get(bpt, prio); \
        default: return nullptr;             \
    }

static EmFn em_lookup(int M, int N, int bpt, bool prio = false) {
    switch (M) {
        case 2: FFCA_N_CASES(2)
        case 3: FFCA_N_CASES(3)
        case 4: FFCA_N_CASES(4)
        default: return nullptr;
    }
}

bool em_supported(int M, int N, int bpt, bool cov) {
    return (cov ? em_cov_lookup(M, N, bpt) : em_lookup(M, N, bpt)) != nullptr;
}

bool em_tail_supported(int M, int N, int bpt, bool cov) {
    return (cov ? em_cov_lookup(M, N, bpt, true) : em_lookup(M, N, bpt, true)) != nullptr;
}

int em_blocks_per_cu(int M, int N, int bpt, int threads, bool cov) {
    EmFn fn = cov ? em_cov_lookup(M, N, bpt) : em_lookup(M, N, bpt);
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, 0) != hipSuccess) return 0;
    return n;
}

// Persistent launch over a mixed batch: every workgroup pulls the next work
// item (one frequency of one mixture, longest first) from a device counter
// and runs it with the (M, N) instantiation it needs. The grid drains when
// the counter passes n_items.
#define FFCA_PERSISTENT_CLASSES(X) X(2, 3) X(2, 4) X(3, 4) X(3, 5) X(4, 5) X(4, 6)

template <int BPT>
__global__ void __launch_bounds__(kResidentBins / BPT) em_persistent_kernel(EmLaunch a) {
    // widest reductions among the classes: Q_m of M = 4, 2NM of (4, 6)
    __shared__ EmSmem<kRedW, 2 * 6 * 4, wave_slots(BPT)> sm;
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1);
        __syncthreads();
        const int i = s_item;
        __syncthreads();
        if (i >= a.n_items) break;
        const WorkItem &it = a.items[i];
        if (*it.status != ST_OK) continue;
        switch (it.M * 16 + it.N) {
#define FFCA_CASE(MM, NN) \
    case MM * 16 + NN: em_item<MM, NN, BPT, false>(it, a.n_iter, a.algo, a.ll_alarm, a.trace_off, sm); break;
            FFCA_PERSISTENT_CLASSES(FFCA_CASE)
#undef FFCA_CASE
            default: break;
        }
    }
}

bool persistent_supported(int M, int N) {
    switch (M * 16 + N) {
#define FFCA_CASE(MM, NN) case MM * 16 + NN: return true;
        FFCA_PERSISTENT_CLASSES(FFCA_CASE)
#undef FFCA_CASE
        default: return false;
    }
}

hipError_t launch_em_persistent(const EmLaunch &a, int threads, int bpt, int grid, hipStream_t s) {
    if (threads < 64 || threads * bpt > kResidentBins || (threads & 63) || !a.queue)
        return hipErrorInvalidValue;
    if (bpt == 4)
        hipLaunchKernelGGL(em_persistent_kernel<4>, dim3(grid), dim3(threads), 0, s, a);
    else if (bpt == 8)
        hipLaunchKernelGGL(em_persistent_kernel<8>, dim3(grid), dim3(threads), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------ wide family
template <> void (*wide_lookup<2>(int, int, bool, bool))(EmLaunch);
template <> void (*wide_lookup<3>(int, int, bool, bool))(EmLaunch);
template <> void (*wide_lookup<4>(int, int, bool, bool))(EmLaunch);
template <> void (*wide_lookup<5>(int, int, bool, bool))(EmLaunch);
template <> void (*wide_lookup<6>(int, int, bool, bool))(EmLaunch);
template <> void (*wide_lookup<7>(int, int, bool, bool))(EmLaunch);
template <> void (*wide_lookup<8>(int, int, bool, bool))(EmLaunch);

static EmFn wide_fn(int M, int N, int bpt, bool prio = false, bool mm = false) {
    switch (M) {
        case 2: return wide_lookup<2>(N, bpt, prio, mm);
        case 3: return wide_lookup<3>(N, bpt, prio, mm);
        case 4: return wide_lookup<4>(N, bpt, prio, mm);
        case 5: return wide_lookup<5>(N, bpt, prio, mm);
        case 6: return wide_lookup<6>(N, bpt, prio, mm);
        case 7: return wide_lookup<7>(N, bpt, prio, mm);
        case 8: return wide_lookup<8>(N, bpt, prio, mm);
        default: return nullptr;
    }
}

bool em_wide_supported(int M, int N, int bpt) { return wide_fn(M, N, bpt) != nullptr; }

bool em_wide_tail_supported(int M, int N, int bpt) { return wide_fn(M, N, bpt, true) != nullptr; }

int em_wide_blocks_per_cu(int M, int N, int bpt, int threads) {
    EmFn fn = wide_fn(M, N, bpt);
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, 0) != hipSuccess) return 0;
    return n;
}

hipError_t launch_em_wide(int M, int N, int bpt, int threads, const EmLaunch &a, int grid,
                          hipStream_t s) {
    EmFn fn = wide_fn(M, N, bpt, a.prio != 0, a.algo == kAlgoMM);
    if (!fn) return hipErrorInvalidValue;
    if (threads < 64 || (threads & 63) || threads * bpt > kWideMaxT || threads > wide_max_threads(bpt))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_em(int M, int N, int bpt, int threads, const EmLaunch &a, int grid,
                     hipStream_t s, bool cov) {
    EmFn fn = cov ? em_cov_lookup(M, N, bpt, a.prio != 0) : em_lookup(M, N, bpt, a.prio != 0);
    if (!fn) return hipErrorInvalidValue;
    if (threads < 64 || threads * bpt > kResidentBins || (threads & 63)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), 0, s, a);
    return hipGetLastError();
}

}  // namespace ffca
