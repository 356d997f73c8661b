// Kernels of the wide IP+EM family (em_wide.hpp) for one microphone count,
// FFCA_WIDE_M, given on the compiler command line; the build compiles this
// file once per M in parallel.
#include "em_wide.hpp"

#ifndef FFCA_WIDE_M
#error "FFCA_WIDE_M must be defined"
#endif

namespace ffca {

template <int M, int N, int BPT>
__global__ void __launch_bounds__(wide_max_threads(BPT)) em_wide_kernel(EmLaunch a) {
    static_assert(wide_max_threads(BPT) / 64 <= kWideWaves, "reduction slots per wave");
    static_assert(wide_region_floats<M, BPT>() <= kWideStage / (wide_max_threads(BPT) / 64), "per-wave scratch");
    __shared__ WideSmem sm;
    const WorkItem &it = a.items[blockIdx.x];
    if (*it.status != ST_OK) return;
    em_wide_item<M, N, BPT>(it, a.n_iter, a.ll_alarm, sm);
}

using WideFn = void (*)(EmLaunch);

template <int M, int N>
static WideFn wide_bpt(int bpt) {
    switch (bpt) {
        case 4: return em_wide_kernel<M, N, 4>;
        case 8: return em_wide_kernel<M, N, 8>;
        default: return nullptr;
    }
}

template <>
void (*wide_lookup<FFCA_WIDE_M>(int N, int bpt))(EmLaunch) {
    constexpr int M = FFCA_WIDE_M;
    switch (N) {
        case 2: return wide_bpt<M, 2>(bpt);
        case 3: return wide_bpt<M, 3>(bpt);
        case 4: return wide_bpt<M, 4>(bpt);
        case 5: return wide_bpt<M, 5>(bpt);
        case 6: return wide_bpt<M, 6>(bpt);
        case 7: return wide_bpt<M, 7>(bpt);
        case 8: return wide_bpt<M, 8>(bpt);
        case 9: return wide_bpt<M, 9>(bpt);
        case 10: return wide_bpt<M, 10>(bpt);
        case 11: return wide_bpt<M, 11>(bpt);
        case 12: return wide_bpt<M, 12>(bpt);
        default: return nullptr;
    }
}

}  // namespace ffca
