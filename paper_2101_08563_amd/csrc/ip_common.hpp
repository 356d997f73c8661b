// Helpers shared by the IP sweeps (ip_sm.hpp, ip_inv.hpp) and the kernels:
// a wavefront maximum and the indexing of the Hermitian upper triangle.
#pragma once

#include "device.hpp"
#include "internal.hpp"

namespace ffca {

__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Index (r, c), r < c, of the p-th strictly upper entry in row-major order.
template <int M>
__device__ __forceinline__ void upper_pair(int p, int &r, int &c) {
    r = 0;
    int rowlen = M - 1;
    while (p >= rowlen) {
        p -= rowlen;
        ++r;
        --rowlen;
    }
    c = r + 1 + p;
}
template <int M>
__device__ __forceinline__ int upper_index(int r, int c) {  // r < c
    return r * (2 * M - r - 1) / 2 + (c - r - 1);
}

}  // namespace ffca
