// Kernels of the wide IP+EM family (em_wide.hpp) for one microphone count,
// FFCA_WIDE_M, given on the compiler command line; the build compiles this
// file once per M in parallel.
#include "em_wide.hpp"

#ifndef FFCA_WIDE_M
#error "FFCA_WIDE_M must be defined"
#endif

namespace ffca {

// PRIO: the tail instance of the tail split (see em_kernel.hip). MM:
// Algorithm 2 (IP+MM) instead of Algorithm 1.
template <int M, int N, int BPT, bool PRIO, bool MM>
__global__ void __launch_bounds__(wide_max_threads(BPT)) em_wide_kernel(EmLaunch a) {
    static_assert(wide_max_threads(BPT) / 64 <= kWideWaves, "reduction slots per wave");
    static_assert(wide_region_floats<M, BPT>() <= kWideStage / (wide_max_threads(BPT) / 64), "per-wave scratch");
    __shared__ WideSmem sm;
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
    const WorkItem &it = a.items[blockIdx.x];
    if (*it.status != ST_OK) return;
    em_wide_item<M, N, BPT, MM>(it, a.n_iter, a.ll_alarm, a.trace_off, sm);
}

using WideFn = void (*)(EmLaunch);

template <int M, int N, bool MM>
static WideFn wide_bpt_algo(int bpt, bool prio) {
    switch (bpt) {
        case 4: return prio ? em_wide_kernel<M, N, 4, true, MM> : em_wide_kernel<M, N, 4, false, MM>;
        case 8: return prio ? em_wide_kernel<M, N, 8, true, MM> : em_wide_kernel<M, N, 8, false, MM>;
        default: return nullptr;
    }
}

template <int M, int N>
static WideFn wide_bpt(int bpt, bool prio, bool mm) {
    return mm ? wide_bpt_algo<M, N, true>(bpt, prio) : wide_bpt_algo<M, N, false>(bpt, prio);
}

template <>
void (*wide_lookup<FFCA_WIDE_M>(int N, int bpt, bool prio, bool mm))(EmLaunch) {
    constexpr int M = FFCA_WIDE_M;
    switch (N) {
        case 2: return wide_bpt<M, 2>(bpt, prio, mm);
        case 3: return wide_bpt<M, 3>(bpt, prio, mm);
        case 4: return wide_bpt<M, 4>(bpt, prio, mm);
        case 5: return wide_bpt<M, 5>(bpt, prio, mm);
        case 6: return wide_bpt<M, 6>(bpt, prio, mm);
        case 7: return wide_bpt<M, 7>(bpt, prio, mm);
        case 8: return wide_bpt<M, 8>(bpt, prio, mm);
        case 9: return wide_bpt<M, 9>(bpt, prio, mm);
        case 10: return wide_bpt<M, 10>(bpt, prio, mm);
        case 11: return wide_bpt<M, 11>(bpt, prio, mm);
        case 12: return wide_bpt<M, 12>(bpt, prio, mm);
        default: return nullptr;
    }
}

}  // namespace ffca
