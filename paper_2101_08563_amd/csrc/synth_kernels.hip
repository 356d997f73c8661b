// Seeded synthetic mixtures on the GPU (benchmark and training data).
//
// The FCA generative model of Sec. III-A with the recipe of the build's
// synthetic workloads: source image c_n(t,f) ~ N_c(0, v_n(t,f) R_n(f)),
// x = sum_n c_n (eq:summodel), with
//   v_n = W_n H_n, rank K, W_n [F,K] and H_n [K,T] with Exp(1) (= Gamma(1,1))
//   entries; R_n(f) = a a^H + delta I, a_m = exp(i theta), theta ~ U[0, 2 pi).
// Random numbers: SplitMix64 (Steele, Lea, Flood 2014) applied to a per-draw
// counter; uniforms take the top 24 bits (in (0, 1)); normals by Box-Muller.
// Holds no FastFCA arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace ffca {

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Uniform in (0, 1) for draw `counter` of stream `stream` under `seed`.
__device__ __forceinline__ float uni(uint64_t seed, uint64_t stream, uint64_t counter) {
    const uint64_t z = mix64(seed + 0x9E3779B97F4A7C15ULL * (counter + 1) + (stream << 56));
    return (static_cast<float>(z >> 40) + 0.5f) * (1.0f / 16777216.0f);
}

constexpr int kMaxGM = 8;

// Per (n, f): W_n(f, :) and the Cholesky factor of R_n(f) = a a^H + delta I.
__global__ void synth_scm_kernel(int F, int M, int N, int K, float delta, uint64_t seed,
                                 float *W /*[N][F][K]*/, float2 *C /*[N][F][M][M]*/) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * F) return;
    const int n = i / F, f = i % F;
    for (int k = 0; k < K; ++k)
        W[(static_cast<size_t>(n) * F + f) * K + k] =
            -logf(uni(seed, 1, (static_cast<uint64_t>(n) * F + f) * K + k));
    float2 a[kMaxGM];
    for (int m = 0; m < M; ++m) {
        const float th = 6.28318530717958647f * uni(seed, 2, (static_cast<uint64_t>(n) * F + f) * M + m);
        float s, c;
        sincosf(th, &s, &c);
        a[m] = make_float2(c, s);
    }
    // Cholesky of R = a a^H + delta I (lower triangular L, R = L L^H), double
    double Lr[kMaxGM][kMaxGM], Li[kMaxGM][kMaxGM];
    for (int r = 0; r < M; ++r)
        for (int c = 0; c <= r; ++c) {
            // R[r][c] = a_r conj(a_c) + delta [r == c]
            double sr = static_cast<double>(a[r].x) * a[c].x + static_cast<double>(a[r].y) * a[c].y;
            double si = static_cast<double>(a[r].y) * a[c].x - static_cast<double>(a[r].x) * a[c].y;
            if (r == c) sr += delta;
            for (int k = 0; k < c; ++k) {
                // subtract L[r][k] conj(L[c][k])
                sr -= Lr[r][k] * Lr[c][k] + Li[r][k] * Li[c][k];
                si -= Li[r][k] * Lr[c][k] - Lr[r][k] * Li[c][k];
            }
            if (r == c) {
                const double d = sqrt(sr);
                Lr[r][r] = d;
                Li[r][r] = 0.0;
            } else {
                Lr[r][c] = sr / Lr[c][c];
                Li[r][c] = si / Lr[c][c];
            }
        }
    float2 *Cn = C + (static_cast<size_t>(n) * F + f) * M * M;
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < M; ++c)
            Cn[r * M + c] = c <= r ? make_float2(static_cast<float>(Lr[r][c]), static_cast<float>(Li[r][c]))
                                   : make_float2(0.f, 0.f);
}

// One thread per (f, t): x(t, f) = sum_n sqrt(v_n(t,f)) L_n(f) z_n(t,f).
__global__ void synth_mix_kernel(int F, int T, int M, int N, int K, uint64_t seed, const float *W,
                                 const float2 *C, float2 *x /*[F][T][M]*/) {
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<size_t>(F) * T) return;
    const int f = static_cast<int>(i / T), t = static_cast<int>(i % T);
    float2 acc[kMaxGM];
    for (int m = 0; m < M; ++m) acc[m] = make_float2(0.f, 0.f);
    for (int n = 0; n < N; ++n) {
        float v = 0.0f;
        for (int k = 0; k < K; ++k) {
            const float h = -logf(uni(seed, 3, (static_cast<uint64_t>(n) * K + k) * T + t));
            v = fmaf(W[(static_cast<size_t>(n) * F + f) * K + k], h, v);
        }
        const float sv = sqrtf(v);
        float2 z[kMaxGM];
        for (int m = 0; m < M; ++m) {
            const uint64_t ctr = ((static_cast<uint64_t>(n) * F + f) * T + t) * M + m;
            const float u1 = uni(seed, 4, ctr), u2 = uni(seed, 5, ctr);
            const float rad = sqrtf(-logf(u1));  // |z|^2 ~ Exp(1): real, imag ~ N(0, 1/2)
            float s, c;
            sincosf(6.28318530717958647f * u2, &s, &c);
            z[m] = make_float2(rad * c, rad * s);
        }
        const float2 *Cn = C + (static_cast<size_t>(n) * F + f) * M * M;
        for (int r = 0; r < M; ++r) {
            float re = 0.f, im = 0.f;
            for (int c = 0; c <= r; ++c) {
                const float2 l = Cn[r * M + c];
                re = fmaf(l.x, z[c].x, fmaf(-l.y, z[c].y, re));
                im = fmaf(l.x, z[c].y, fmaf(l.y, z[c].x, im));
            }
            acc[r].x = fmaf(sv, re, acc[r].x);
            acc[r].y = fmaf(sv, im, acc[r].y);
        }
    }
    for (int m = 0; m < M; ++m) x[i * M + m] = acc[m];
}

}  // namespace

hipError_t launch_synth(float2 *x, int F, int T, int M, int N, int K, float delta, uint64_t seed,
                        float *W, float2 *C, hipStream_t s) {
    if (M < 1 || M > kMaxGM || N < 1 || K < 1 || F < 1 || T < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(synth_scm_kernel, dim3((N * F + 127) / 128), dim3(128), 0, s, F, M, N, K, delta,
                       seed, W, C);
    const size_t bins = static_cast<size_t>(F) * T;
    hipLaunchKernelGGL(synth_mix_kernel, dim3(static_cast<unsigned>((bins + 255) / 256)), dim3(256), 0, s, F,
                       T, M, N, K, seed, W, C, x);
    return hipGetLastError();
}

}  // namespace ffca
