// IP+EM kernels of the piecewise stationary model (Sec. VI): every bin is a
// block of B frames whose block covariance Xhat_j replaces x_j x_j^H in
// Algorithms 1 and 2. Same per-item body as em_kernel.hip (em_item.hpp with
// COV = true); a separate translation unit so the two families compile in
// parallel.
#include "em_item.hpp"

namespace ffca {

// PRIO: the tail instance of the tail split, as in em_kernel.hip.
template <int M, int N, int BPT, bool PRIO>
__global__ void __launch_bounds__(kResidentBins / BPT) em_cov_kernel(EmLaunch a) {
    __shared__ EmSmem<M * M * M, 2 * N * M, wave_slots(BPT)> sm;
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
    const WorkItem &it = a.items[blockIdx.x];
    if (*it.status != ST_OK) return;  // frozen after an earlier failure
    em_item<M, N, BPT, true>(it, a.n_iter, a.algo, a.ll_alarm, a.trace_off, sm);
}

template <int M, int N>
static EmFn cov_bpt(int bpt, bool prio) {
    switch (bpt) {
        case 2: return prio ? nullptr : em_cov_kernel<M, N, 2, false>;
        case 4: return prio ? em_cov_kernel<M, N, 4, true> : em_cov_kernel<M, N, 4, false>;
        case 8: return prio ? em_cov_kernel<M, N, 8, true> : em_cov_kernel<M, N, 8, false>;
        case 16: return prio ? nullptr : em_cov_kernel<M, N, 16, false>;
        default: return nullptr;
    }
}

#define FFCA_COV_N(M)                   \
    switch (N) {                        \
        case 2: return cov_bpt<M, 2>(bpt, prio); \
        case 3: return cov_bpt<M, 3>(bpt, prio); \
        case 4: return cov_bpt<M, 4>(bpt, prio); \
        case 5: return cov_bpt<M, 5>(bpt, prio); \
        case 6: return cov_bpt<M, 6>(bpt, prio); \
        case 7: return cov_bpt<M, 7>(bpt, prio); \
        case 8: return cov_bpt<M, 8>(bpt, prio); \
        default: return nullptr;        \
    }

EmFn em_cov_lookup(int M, int N, int bpt, bool prio) {
    switch (M) {
        case 2: FFCA_COV_N(2)
        case 3: FFCA_COV_N(3)
        case 4: FFCA_COV_N(4)
        default: return nullptr;
    }
}

}  // namespace ffca
