// FastMNMF launch interface shared by mnmf_kernels.hip and the runtime.
#pragma once

#include <hip/hip_runtime.h>

namespace ffca {

constexpr int kMnmfKMax = 32;  // NMF bases per source
constexpr int kMnmfKC = 8;     // bases reduced together in the T update
constexpr int kMnmfNMax = 6;   // sources
constexpr int kMnmfFChunk = 32;  // frequencies per partial sum of the V rule

struct MnmfLaunch {
    const float2 *x;   // [F][T][M]
    double2 *P;        // [F][M][M]
    float *lam;        // [F][N][M]
    float *tp;         // [F][K][N] spectral patterns t_{ikn}
    const float *va;   // [K][N][T] activations v_{jkn} (frames contiguous)
    float *G, *E;      // [F][T][N] V-rule terms
    double *ll_trace;  // [F][cap]
    int cap;
    double *ldet;      // [F] ln|det P|^2 of the current P
    int *status;       // [F]
    int F, T, K;
    int iter;          // iteration index; the LL of the current state goes to iter - 1
    int ll_only;       // 1: only that LL (evaluation after the last iteration)
};

bool mnmf_supported(int M, int N, int bpt);
hipError_t launch_mnmf_freq(int M, int N, int bpt, int threads, const MnmfLaunch &a, hipStream_t s);
hipError_t launch_mnmf_v(const float *G, const float *E, const float *tp, float *part, float *va, int F, int T,
                         int N, int K, int fchunk, int *flag, hipStream_t s);
// out[c][r] = in[r][c]: activations between the ABI layout [T][K][N] and [K][N][T]
hipError_t launch_transpose(const float *in, float *out, int R, int C, hipStream_t s);
hipError_t launch_mnmf_h(const float *tp, const float *va, float *h, int F, int T, int N, int K, hipStream_t s);

}  // namespace ffca
