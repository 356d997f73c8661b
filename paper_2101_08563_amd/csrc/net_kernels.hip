// Kernels of the learned warm start: whitened log-power features, a 1-D
// convolutional network over time applied to every frequency with shared
// weights (BF16 operands on the 16x16x16 MFMA, FP32 accumulation), its
// backward pass, the permutation-invariant loss, training targets from
// converged FastFCA fits, and AdamW.
//
// Activation tensors are FP32 [S][C][T] (S sequences = frequencies of one or
// more mixtures, C channels, T frames). A convolution with kernel size KS and
// "same" zero padding R = KS / 2 is the GEMM
//   Y[co][t] = sum_{kk} W[co][kk] X~[kk][t],  kk = k * Cin + ci,
//   X~[kk][t] = X[ci][t + k - R],
// whose weight operand is stored as BF16 [Cout][Kp] (Kp = Cin*KS rounded up
// to 16, zero padded).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "internal.hpp"

namespace ffca {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

constexpr int kTile = 64;      // frames per workgroup
constexpr int kMaxC = 64;      // channels
constexpr int kMaxKp = 320;    // 64 channels x kernel 5

// ------------------------------------------------------------------ weights
// GEMM column order is k-major: kk = k * Cin + ci.
// fp32 master W (row co at W + co*ldw holding entries ci*KS + k) -> bf16
// Wb[Cout][Kp] with Wb[co][k*Cin + ci] = W[co][ci*KS + k]; if transpose_flip,
// the operand of the data-gradient convolution (Cin rows, input channels co):
// Wt[ci][k*Cout + co] = W[co][ci*KS + KS-1-k].
__global__ void pack_weights_kernel(const float *W, int ldw, int Cout, int Cin, int KS, int Kp,
                                    int transpose_flip, uint16_t *Wb) {
    const int rows = transpose_flip ? Cin : Cout;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * Kp) return;
    const int r = i / Kp, kk = i % Kp;
    float v = 0.0f;
    if (!transpose_flip) {
        if (kk < Cin * KS) {
            const int k = kk / Cin, ci = kk % Cin;
            v = W[static_cast<size_t>(r) * ldw + ci * KS + k];
        }
    } else {
        if (kk < Cout * KS) {
            const int k = kk / Cout, co = kk % Cout;
            v = W[static_cast<size_t>(co) * ldw + r * KS + (KS - 1 - k)];
        }
    }
    Wb[i] = f2bf(v);
}

// ------------------------------------------------------------------ forward
// mode 0: Y = pre; 1: Y = relu(pre); 2: Y = Res + relu(pre); 3: Y = Res + pre;
// pre = bias[co] + conv. Pre (optional) receives pre.
// Grid (ceil(T / kChunk), S), 256 threads. Wave w owns output rows
// 16w..16w+15 and keeps their weight fragments in registers for the whole
// chunk; each 64-frame tile of X is staged in LDS as bf16 [t][ci] so a B
// fragment (4 consecutive kk = 4 consecutive channels at one tap) is one
// 8-byte LDS read when Cin is a multiple of 4.
constexpr int kChunk = 256;
constexpr int kMaxKb = kMaxKp / 16;

template <int KS>
__global__ void __launch_bounds__(256) conv_fwd_kernel(const float *X, int Cin, const uint16_t *Wb, int Kp,
                                                       const float *bias, int Cout, float *Y, int T,
                                                       int mode, const float *Res, float *Pre) {
    constexpr int R = KS / 2;
    constexpr int XW = kTile + KS - 1;
    __shared__ __align__(16) uint16_t xs[XW][kMaxC + 4];
    const int s = blockIdx.y;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int Kreal = Cin * KS;
    const int nkb = Kp / 16;
    const bool active = 16 * w < Cout;
    // weight fragments of this wave's 16 rows
    bf16x4 afrag[kMaxKb];
#pragma unroll
    for (int kb = 0; kb < kMaxKb; ++kb) {
        bf16x4 a = bf16x4{0, 0, 0, 0};
        if (kb < nkb && active && 16 * w + li < Cout) {
            const uint16_t *src = Wb + static_cast<size_t>(16 * w + li) * Kp + kb * 16 + 4 * lq;
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = static_cast<short>(src[q]);
        }
        afrag[kb] = a;
    }
    const float *Xs = X + static_cast<size_t>(s) * Cin * T;
    const int tbeg = blockIdx.x * kChunk;
    const int tend = min(T, tbeg + kChunk);
    const bool vec = (Cin % 4) == 0;
    // X tiles are staged through registers with every load of a tile issued
    // at once, before the first LDS store
    constexpr int kStage = (kMaxC * XW + 255) / 256;
    for (int t0 = tbeg; t0 < tend; t0 += kTile) {
        __syncthreads();
        {
            float sv[kStage];
#pragma unroll
            for (int r = 0; r < kStage; ++r) {
                const int i = tid + 256 * r;
                const int ci = i / XW, tt = i % XW;
                const int t = t0 + tt - R;
                sv[r] = (i < Cin * XW && t >= 0 && t < T) ? Xs[static_cast<size_t>(ci) * T + t] : 0.0f;
            }
#pragma unroll
            for (int r = 0; r < kStage; ++r) {
                const int i = tid + 256 * r;
                if (i < Cin * XW) xs[i % XW][i / XW] = f2bf(sv[r]);
            }
        }
        __syncthreads();
        if (!active) continue;
        f32x4 acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < kMaxKb; ++kb) {
            if (kb >= nkb) continue;
            const int kk0 = kb * 16 + 4 * lq;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                bf16x4 b;
                if (vec) {
                    if (kk0 < Kreal) {
                        const int k = kk0 / Cin, ci = kk0 - k * Cin;
                        b = *reinterpret_cast<const bf16x4 *>(&xs[16 * j + li + k][ci]);
                    } else {
                        b = bf16x4{0, 0, 0, 0};
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int kk = kk0 + q;
                        uint16_t v = 0;
                        if (kk < Kreal) {
                            const int k = kk / Cin, ci = kk - k * Cin;
                            v = xs[16 * j + li + k][ci];
                        }
                        b[q] = static_cast<short>(v);
                    }
                }
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(afrag[kb], b, acc[j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = t0 + 16 * j + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int co = 16 * w + 4 * lq + v;
                if (co < Cout && t < T) {
                    const size_t o = (static_cast<size_t>(s) * Cout + co) * T + t;
                    const float pre = acc[j][v] + (bias ? bias[co] : 0.0f);
                    float y;
                    if (mode == 0)
                        y = pre;
                    else if (mode == 1)
                        y = fmaxf(pre, 0.0f);
                    else if (mode == 2)
                        y = Res[o] + fmaxf(pre, 0.0f);
                    else
                        y = Res[o] + pre;
                    Y[o] = y;
                    if (Pre) Pre[o] = pre;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ fused inference
// The whole forward pass for one sequence and one tile of kFT output frames
// in one workgroup, with the activations in LDS: the kernel-5 input layer,
// the L residual layers and the 1x1 head. Each kernel-5 layer narrows the
// valid frames by 2 on each side, so the tile is computed over kFT + 4 (L + 1)
// input frames (a 2 (L + 1)-frame halo each side) and rows whose frame lies
// outside [0, T) are held at zero, which is the "same" zero padding of the
// layer-by-layer convolutions. The convolutions use the same BF16 fragments,
// the same k order and the same MFMA sequence as conv_fwd_kernel; the
// residual stream stays FP32 (hf), and the BF16 copy that feeds the MFMAs
// alternates between two buffers, so a wave stores each 16-frame block of a
// layer as soon as it is done, with one barrier per layer. The LDS buffers
// are sized for the instance's C, so narrower networks keep more workgroups
// per CU. The head (N outputs) and the per-tile sums of h_L over frames are
// plain FP32; the tile sums are combined in order by pool_tiles_kernel.
constexpr int kFT = 64;                                // output frames per tile
constexpr int kFMaxL = 8;                              // residual layers
constexpr int kFMaxN = 8;                              // head outputs
constexpr int kFRows = kFT + 4 * (kFMaxL + 1) + 16;    // input rows + overrun of the last 16-row block

struct FusedNetArgs {
    const float *feat;  // [S][M][T]
    float *lv;          // [S][N][T]
    float *part;        // [S][ntiles][C]
    const uint16_t *W[kFMaxL + 1];
    const float *b[kFMaxL + 1];
    const float *Wv;    // [N][ldv], FP32 head weights
    const float *bv;    // [N]
    int S, M, T, C, L, N, Kp0, ldv, ntiles;
};

template <int C>
__global__ void __launch_bounds__(256) net_fused_fwd_kernel(FusedNetArgs a) {
    __shared__ __align__(16) float hf[kFRows][C + 1];
    __shared__ __align__(16) uint16_t hb[2][kFRows][C + 4];  // layer input / output, alternating
    __shared__ __align__(16) uint16_t fb[kFRows][4];
    __shared__ float wvs[kFMaxN][C];
    __shared__ float bs[kFMaxL + 1][C];
    const int s = blockIdx.y, tile = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int L = a.L, T = a.T, M = a.M;
    const int H = 2 * (L + 1);
    const int W0 = kFT + 2 * H;
    const int t0 = tile * kFT;
    const int fr0 = t0 - H;  // frame of row 0
    static_assert((2 * kFRows * (C + 4) * 2) % 16 == 0, "16-byte clears");
    for (int i = tid; i < 2 * kFRows * (C + 4) * 2 / 16; i += 256)
        reinterpret_cast<uint4 *>(&hb[0][0][0])[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int i = tid; i < kFRows * 2; i += 256) reinterpret_cast<uint32_t *>(&fb[0][0])[i] = 0u;
    for (int i = tid; i < a.N * C; i += 256) wvs[i / C][i % C] = a.Wv[static_cast<size_t>(i / C) * a.ldv + i % C];
    for (int i = tid; i < (L + 1) * C; i += 256) bs[i / C][i % C] = a.b[i / C][i % C];
    __syncthreads();
    for (int i = tid; i < M * W0; i += 256) {
        const int ci = i / W0, r = i % W0;
        const int t = fr0 + r;
        fb[r][ci] = f2bf((t >= 0 && t < T) ? a.feat[(static_cast<size_t>(s) * M + ci) * T + t] : 0.0f);
    }
    __syncthreads();

    const bool act = 16 * w < C;  // wave w owns channels 16 w .. 16 w + 15
    // output rows [lo, hi) of a layer: activation, residual, zero padding
    // (res: the residual values of the lane's four outputs, zero for layer 0)
    auto store = [&](int l, int j, int lo, int hi, const f32x4 &c, const f32x4 &res,
                     uint16_t (*out)[C + 4]) {
        const int r = lo + 16 * j + li;
        if (r >= hi) return;
        const int t = fr0 + r;
        const bool in = t >= 0 && t < T;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int co = 16 * w + 4 * lq + v;
            const float val = in ? res[v] + fmaxf(c[v] + bs[l][co], 0.0f) : 0.0f;
            hf[r][co] = val;
            out[r][co] = f2bf(val);
        }
    };

    // this wave's 16 weight rows of a residual layer, every fragment load in
    // flight at once; the next layer's are loaded while this one computes
    constexpr int nkb = 5 * C / 16;
    auto load_frags = [&](int l, bf16x4 (&af)[nkb]) {
        const uint16_t *Wl = a.W[l] + static_cast<size_t>(16 * w + li) * (5 * C) + 4 * lq;
#pragma unroll
        for (int kb = 0; kb < nkb; ++kb) af[kb] = *reinterpret_cast<const bf16x4 *>(Wl + 16 * kb);
    };
    bf16x4 afn[nkb];
    if (act && L >= 1) load_frags(1, afn);

    // layer 0: M input channels, one or two 16-wide k blocks, gathered from fb
    if (act) {
        const int Kp = a.Kp0;
        const uint16_t *Wl = a.W[0] + static_cast<size_t>(16 * w + li) * Kp + 4 * lq;
        const int lo = 2, hi = W0 - 2;
        const int nblk = (hi - lo + 15) / 16;
        // the lane's (tap, channel) of each of its k entries: k blocks of 16,
        // at most two since 5 M <= 20
        int gk[2][4], gc[2][4];
        bool gv[2][4];
        bf16x4 af0[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            af0[kb] = kb < Kp / 16 ? *reinterpret_cast<const bf16x4 *>(Wl + 16 * kb) : bf16x4{0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = 16 * kb + 4 * lq + q;
                gv[kb][q] = kk < 5 * M;
                gk[kb][q] = gv[kb][q] ? kk / M : 0;
                gc[kb][q] = gv[kb][q] ? kk - (kk / M) * M : 0;
            }
        }
        for (int j = 0; j < nblk; ++j) {
            f32x4 c = f32x4{0.f, 0.f, 0.f, 0.f};
            const int rb = lo + 16 * j + li - 2;
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                if (kb >= Kp / 16) break;
                bf16x4 bq;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    bq[q] = gv[kb][q] ? static_cast<short>(fb[rb + gk[kb][q]][gc[kb][q]]) : 0;
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af0[kb], bq, c, 0, 0, 0);
            }
            store(0, j, lo, hi, c, f32x4{0.f, 0.f, 0.f, 0.f}, hb[0]);
        }
    }
    __syncthreads();

    // residual layers: input hb[(l + 1) & 1], output hb[l & 1]
    for (int l = 1; l <= L; ++l) {
        uint16_t (*in)[C + 4] = hb[(l + 1) & 1];
        uint16_t (*out)[C + 4] = hb[l & 1];
        const int lo = 2 * (l + 1), hi = W0 - 2 * (l + 1);
        const int nblk = (hi - lo + 15) / 16;
        if (act) {
            bf16x4 af[nkb];
#pragma unroll
            for (int kb = 0; kb < nkb; ++kb) af[kb] = afn[kb];
            if (l < L) load_frags(l + 1, afn);
#pragma unroll 1
            for (int j = 0; j < nblk; ++j) {
                const int rb = lo + 16 * j + li - 2;  // input row of tap 0
                // every B fragment of the block read before the first MFMA
                bf16x4 bq[nkb];
#pragma unroll
                for (int kb = 0; kb < nkb; ++kb) {
                    const int kk0 = 16 * kb + 4 * lq;
                    const int k = kk0 / C, ci = kk0 - k * C;
                    bq[kb] = *reinterpret_cast<const bf16x4 *>(&in[rb + k][ci]);
                }
                // the residual of the lane's outputs (rows past the layer read a
                // row inside the buffer and are not stored)
                f32x4 res;
                {
                    const int r = min(lo + 16 * j + li, kFRows - 1);
#pragma unroll
                    for (int v = 0; v < 4; ++v) res[v] = hf[r][16 * w + 4 * lq + v];
                }
                __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the MFMA chains
                // two accumulators (even and odd k blocks) so that consecutive
                // MFMAs do not wait on each other
                f32x4 c0 = f32x4{0.f, 0.f, 0.f, 0.f}, c1 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb + 1 < nkb; kb += 2) {
                    c0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[kb], bq[kb], c0, 0, 0, 0);
                    c1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[kb + 1], bq[kb + 1], c1, 0, 0, 0);
                }
                if constexpr (nkb % 2) c0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[nkb - 1], bq[nkb - 1], c0, 0, 0, 0);
                const f32x4 c = c0 + c1;
                store(l, j, lo, hi, c, res, out);
            }
        }
        __syncthreads();
    }
    // head: log v[n][t] = bv[n] + sum_c Wv[n][c] h_L[t][c]
    for (int q = tid; q < a.N * kFT; q += 256) {
        const int n = q / kFT, i = q - n * kFT;
        const int t = t0 + i;
        if (t < T) {
            float y = a.bv[n];
#pragma unroll
            for (int c = 0; c < C; ++c) y = fmaf(wvs[n][c], hf[H + i][c], y);
            a.lv[(static_cast<size_t>(s) * a.N + n) * T + t] = y;
        }
    }
    // this tile's sum of h_L over its frames, per channel
    for (int c = tid; c < C; c += 256) {
        float sum = 0.0f;
        for (int i = 0; i < kFT && t0 + i < T; ++i) sum += hf[H + i][c];
        a.part[(static_cast<size_t>(s) * a.ntiles + tile) * C + c] = sum;
    }
}

// pooled[s][c] = (1/T) sum over tiles in order of part[s][tile][c]
__global__ void pool_tiles_kernel(const float *part, int S, int ntiles, int C, int T, float *pooled) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * C) return;
    const int s = i / C, c = i - s * C;
    float sum = 0.0f;
    for (int k = 0; k < ntiles; ++k) sum += part[(static_cast<size_t>(s) * ntiles + k) * C + c];
    pooled[i] = sum / static_cast<float>(T);
}

// ------------------------------------------------------------------ weight gradient
// dW[co][ci*KS + k] += sum_t G[s][co][t] X[s][ci][t + k - R];  db[co] += sum_t G[s][co][t].
// Computed as the GEMM over kk = k * Cin + ci. Grid (ceil(T / kChunk), S): a
// workgroup accumulates its frame chunk in registers (wave w owns a quarter of
// the (co, kk) tiles) and adds the result once with float atomics into FP32
// dW (row stride Kp, the float master's layout) and db [Cout].
constexpr int kBwTiles = 20;  // (64/16) * (320/16) / 4 waves
template <int KS>
__global__ void __launch_bounds__(256) conv_bwdw_kernel(const float *G, int Cout, const float *X, int Cin,
                                                        int Kp, int T, float *dW, float *db) {
    constexpr int R = KS / 2;
    constexpr int XW = kTile + KS - 1;
    __shared__ __align__(16) uint16_t xs[kMaxC][XW + 3];
    __shared__ __align__(16) uint16_t gs[kMaxC][kTile + 4];
    const int s = blockIdx.y;
    const int tid = threadIdx.x;
    const float *Xs = X + static_cast<size_t>(s) * Cin * T;
    const float *Gs = G + static_cast<size_t>(s) * Cout * T;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int Kreal = Cin * KS;
    const int n_co = (Cout + 15) / 16, n_kk = Kp / 16;
    const int ntile = n_co * n_kk;
    f32x4 acc[kBwTiles];
#pragma unroll
    for (int i = 0; i < kBwTiles; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.0f;
    const int tbeg = blockIdx.x * kChunk;
    const int tend = min(T, tbeg + kChunk);
    for (int t0 = tbeg; t0 < tend; t0 += kTile) {
        __syncthreads();
        for (int i = tid; i < Cin * XW; i += 256) {
            const int ci = i / XW, tt = i % XW;
            const int t = t0 + tt - R;
            xs[ci][tt] = f2bf((t >= 0 && t < T) ? Xs[static_cast<size_t>(ci) * T + t] : 0.0f);
        }
        for (int i = tid; i < kMaxC * kTile; i += 256) {
            const int co = i / kTile, tt = i % kTile;
            const int t = t0 + tt;
            gs[co][tt] = f2bf((co < Cout && t < T) ? Gs[static_cast<size_t>(co) * T + t] : 0.0f);
        }
        __syncthreads();
        if (tid < Cout)
            for (int tt = 0; tt < kTile && t0 + tt < T; ++tt) bacc += Gs[static_cast<size_t>(tid) * T + t0 + tt];
#pragma unroll
        for (int i = 0; i < kBwTiles; ++i) {
            const int tile = w + 4 * i;
            if (tile >= ntile) continue;
            const int cot = tile / n_kk, kkt = tile % n_kk;
            const int kk = 16 * kkt + li;
            const int k = kk / Cin, ci = kk - k * Cin;
#pragma unroll
            for (int tc = 0; tc < kTile / 16; ++tc) {
                const int tb = 16 * tc + 4 * lq;
                const bf16x4 a = *reinterpret_cast<const bf16x4 *>(&gs[16 * cot + li][tb]);
                bf16x4 b;
#pragma unroll
                for (int q = 0; q < 4; ++q) b[q] = kk < Kreal ? static_cast<short>(xs[ci][tb + q + k]) : 0;
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i], 0, 0, 0);
            }
        }
    }
    if (tid < Cout && db) atomicAdd(db + tid, bacc);
#pragma unroll
    for (int i = 0; i < kBwTiles; ++i) {
        const int tile = w + 4 * i;
        if (tile >= ntile) continue;
        const int cot = tile / n_kk, kkt = tile % n_kk;
        const int kk = 16 * kkt + li;
        const int k = kk / Cin, ci = kk - k * Cin;  // stored in the master's order ci*KS + k
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int co = 16 * cot + 4 * lq + v;
            if (co < Cout && kk < Kreal) atomicAdd(dW + static_cast<size_t>(co) * Kp + ci * KS + k, acc[i][v]);
        }
    }
}

// ------------------------------------------------------------------ elementwise
// G' = G * (Pre > 0)
__global__ void relu_grad_kernel(const float *G, const float *Pre, float *out, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        out[i] = Pre[i] > 0.0f ? G[i] : 0.0f;
}

// pooled[s][c] = (1/T) sum_t H[s][c][t]; one workgroup per (s, c)
__global__ void mean_t_kernel(const float *H, int T, float *pooled) {
    const size_t sc = blockIdx.x;
    const float *h = H + sc * T;
    float a = 0.0f;
    for (int t = threadIdx.x; t < T; t += blockDim.x) a += h[t];
    a = wave_sum(a);
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) pooled[sc] = ((red[0] + red[1]) + (red[2] + red[3])) / static_cast<float>(T);
}

// dH[s][c][t] += dpooled[s][c] / T
__global__ void mean_t_bwd_kernel(const float *dpooled, int T, float *dH, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        dH[i] += dpooled[i / T] / static_cast<float>(T);
}

// out[s][j] = b[j] + sum_c Wl[j][c] in[s][c]   (one thread per (s, j))
__global__ void linear_fwd_kernel(const float *in, int S, int C, const float *Wl, const float *bl, int J,
                                  float *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * J) return;
    const int s = i / J, j = i % J;
    float a = bl[j];
    for (int c = 0; c < C; ++c) a = fmaf(Wl[j * C + c], in[s * C + c], a);
    out[i] = a;
}

// dWl[j][c] += sum_s g[s][j] in[s][c]; dbl[j] += sum_s g[s][j]; din[s][c] = sum_j Wl[j][c] g[s][j]
__global__ void linear_bwd_kernel(const float *in, int S, int C, const float *Wl, int J, const float *g,
                                  float *dWl, float *dbl, float *din) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < J * C) {
        const int j = i / C, c = i % C;
        float a = 0.0f;
        for (int s = 0; s < S; ++s) a = fmaf(g[s * J + j], in[s * C + c], a);
        dWl[i] += a;
    }
    if (i < J) {
        float a = 0.0f;
        for (int s = 0; s < S; ++s) a += g[s * J + i];
        dbl[i] += a;
    }
    if (i < S * C) {
        const int s = i / C, c = i % C;
        float a = 0.0f;
        for (int j = 0; j < J; ++j) a = fmaf(Wl[j * C + c], g[s * J + j], a);
        din[i] = a;
    }
}

// ------------------------------------------------------------------ PIT loss
// Per sequence s (one workgroup): for every order pi of the N sources,
//   L(pi) = mean_{n,t} (lv[s][pi(n)][t] - tv[s][n][t])^2
//         + wl * mean_{n,m} (ll[s][pi(n)][m] - tl[s][n][m])^2,
// loss[s] = min_pi L(pi); the gradient flows through the minimizing order.
// Orders are enumerated in lexicographic order; ties keep the first.
constexpr int kPitMaxN = 4;
__global__ void pit_loss_kernel(const float *lv, const float *tv, const float *ll, const float *tl, int N,
                                int M, int T, float wl, float *loss, int *perm_out, float *glv, float *gll) {
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    __shared__ float Sv[kPitMaxN][kPitMaxN];
    __shared__ float red[4];
    const float *lvs = lv + static_cast<size_t>(s) * N * T;
    const float *tvs = tv + static_cast<size_t>(s) * N * T;
    // pairwise sums over t: Sv[a][b] = sum_t (lv[a] - tv[b])^2
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            float acc = 0.0f;
            for (int t = tid; t < T; t += blockDim.x) {
                const float d = lvs[a * T + t] - tvs[b * T + t];
                acc = fmaf(d, d, acc);
            }
            acc = wave_sum(acc);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) Sv[a][b] = (red[0] + red[1]) + (red[2] + red[3]);
            __syncthreads();
        }
    __shared__ int best_perm[kPitMaxN];
    if (tid == 0) {
        int p[kPitMaxN];
        for (int n = 0; n < N; ++n) p[n] = n;
        float best = INFINITY;
        int bp[kPitMaxN];
        for (;;) {
            float L = 0.0f, Ll = 0.0f;
            for (int n = 0; n < N; ++n) {
                L += Sv[p[n]][n];
                for (int m = 0; m < M; ++m) {
                    const float d = ll[(static_cast<size_t>(s) * N + p[n]) * M + m] - tl[(static_cast<size_t>(s) * N + n) * M + m];
                    Ll = fmaf(d, d, Ll);
                }
            }
            const float tot = L / static_cast<float>(N * T) + wl * Ll / static_cast<float>(N * M);
            if (tot < best) {
                best = tot;
                for (int n = 0; n < N; ++n) bp[n] = p[n];
            }
            // next lexicographic permutation
            int i = N - 2;
            while (i >= 0 && p[i] > p[i + 1]) --i;
            if (i < 0) break;
            int j = N - 1;
            while (p[j] < p[i]) --j;
            int tmp = p[i];
            p[i] = p[j];
            p[j] = tmp;
            for (int a = i + 1, b = N - 1; a < b; ++a, --b) {
                tmp = p[a];
                p[a] = p[b];
                p[b] = tmp;
            }
        }
        for (int n = 0; n < N; ++n) best_perm[n] = bp[n];
        loss[s] = best;
        if (perm_out)
            for (int n = 0; n < N; ++n) perm_out[s * N + n] = bp[n];
    }
    __syncthreads();
    if (glv) {
        const float sc = 2.0f / static_cast<float>(N * T);
        for (int n = 0; n < N; ++n) {
            const int a = best_perm[n];
            for (int t = tid; t < T; t += blockDim.x)
                glv[(static_cast<size_t>(s) * N + a) * T + t] = sc * (lvs[a * T + t] - tvs[n * T + t]);
        }
    }
    if (gll && tid < N * M) {
        const int n = tid / M, m = tid % M;
        const int a = best_perm[n];
        gll[(static_cast<size_t>(s) * N + a) * M + m] =
            wl * 2.0f / static_cast<float>(N * M) *
            (ll[(static_cast<size_t>(s) * N + a) * M + m] - tl[(static_cast<size_t>(s) * N + n) * M + m]);
    }
}

// ------------------------------------------------------------------ AdamW
// Decoupled weight decay (Loshchilov and Hutter): p <- p - lr (mhat/(sqrt(vhat)+eps) + wd p).
__global__ void adamw_kernel(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1,
                             float b2, float eps, float wd, float bc1, float bc2, float gscale) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const float gi = g[i] * gscale;
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / bc1, vh = vi / bc2;
        p[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
    }
}

// ------------------------------------------------------------------ features
// One workgroup per frequency item (x [T][M] of one mixture frequency):
//   C = (1/T) sum_t x_t x_t^H, P0 = C^{-1/2} (Hermitian inverse square root by
//   the coupled Newton-Schulz iteration in double precision), feat[m][t] =
//   ln(|(P0^H x_t)_m|^2 + eps) - mean_t(...). Writes P0 [M][M] (complex128) and
//   feat [M][T] (float). M <= 4, a template argument so that the small
//   matrices stay in registers.
constexpr int kFeatMaxM = 4;
template <int M>
__global__ void __launch_bounds__(256) features_kernel(const float2 *x, int T, float eps, double2 *P0,
                                                       float *feat) {
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    const float2 *xf = x + static_cast<size_t>(f) * T * M;
    __shared__ double red[4][M * M * 2];
    __shared__ double2 Ps[M * M];
    __shared__ float mred[4][M];
    // covariance (double accumulation)
    double acc[M * M * 2];
    for (int i = 0; i < M * M * 2; ++i) acc[i] = 0.0;
    for (int t = tid; t < T; t += blockDim.x) {
        for (int r = 0; r < M; ++r) {
            const float2 a = xf[static_cast<size_t>(t) * M + r];
            for (int c = 0; c < M; ++c) {
                const float2 b = xf[static_cast<size_t>(t) * M + c];
                acc[(r * M + c) * 2] += static_cast<double>(a.x) * b.x + static_cast<double>(a.y) * b.y;
                acc[(r * M + c) * 2 + 1] += static_cast<double>(a.y) * b.x - static_cast<double>(a.x) * b.y;
            }
        }
    }
    for (int i = 0; i < M * M * 2; ++i) {
        const double v = wave_sum(acc[i]);
        if ((tid & 63) == 0) red[tid >> 6][i] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double Cr[M][M], Ci[M][M];
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) {
                const int i = (r * M + c) * 2;
                Cr[r][c] = ((red[0][i] + red[1][i]) + (red[2][i] + red[3][i])) / T;
                Ci[r][c] = ((red[0][i + 1] + red[1][i + 1]) + (red[2][i + 1] + red[3][i + 1])) / T;
            }
        // C^{-1/2} by the coupled Newton-Schulz iteration (Higham, Functions of
        // Matrices, Sec. 6.3): with A = C / ||C||_F (eigenvalues in (0, 1]),
        // Y0 = A, Z0 = I, S = (3I - Z Y)/2, Y <- Y S, Z <- S Z; Z -> A^{-1/2}.
        double fn = 0.0;
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) fn += Cr[r][c] * Cr[r][c] + Ci[r][c] * Ci[r][c];
        fn = sqrt(fn);
        double Yr[M][M], Yi[M][M];
        double Zr[M][M], Zi[M][M];
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) {
                Yr[r][c] = Cr[r][c] / fn;
                Yi[r][c] = Ci[r][c] / fn;
                Zr[r][c] = r == c ? 1.0 : 0.0;
                Zi[r][c] = 0.0;
            }
        for (int it = 0; it < 100; ++it) {
            double Sr[M][M], Si[M][M];
            double dev = 0.0;
            for (int r = 0; r < M; ++r)
                for (int c = 0; c < M; ++c) {
                    double zr = 0.0, zi = 0.0;  // (Z Y)[r][c]
                    for (int k = 0; k < M; ++k) {
                        zr += Zr[r][k] * Yr[k][c] - Zi[r][k] * Yi[k][c];
                        zi += Zr[r][k] * Yi[k][c] + Zi[r][k] * Yr[k][c];
                    }
                    const double er = (r == c ? 1.0 : 0.0) - zr;
                    dev += er * er + zi * zi;
                    Sr[r][c] = 0.5 * ((r == c ? 3.0 : 0.0) - zr);
                    Si[r][c] = -0.5 * zi;
                }
            if (dev < 1e-28) break;
            double Yn_r[M][M], Yn_i[M][M];
            double Zn_r[M][M], Zn_i[M][M];
            for (int r = 0; r < M; ++r)
                for (int c = 0; c < M; ++c) {
                    double yr = 0.0, yi = 0.0, zr = 0.0, zi = 0.0;
                    for (int k = 0; k < M; ++k) {
                        yr += Yr[r][k] * Sr[k][c] - Yi[r][k] * Si[k][c];
                        yi += Yr[r][k] * Si[k][c] + Yi[r][k] * Sr[k][c];
                        zr += Sr[r][k] * Zr[k][c] - Si[r][k] * Zi[k][c];
                        zi += Sr[r][k] * Zi[k][c] + Si[r][k] * Zr[k][c];
                    }
                    Yn_r[r][c] = yr;
                    Yn_i[r][c] = yi;
                    Zn_r[r][c] = zr;
                    Zn_i[r][c] = zi;
                }
            for (int r = 0; r < M; ++r)
                for (int c = 0; c < M; ++c) {
                    Yr[r][c] = Yn_r[r][c];
                    Yi[r][c] = Yn_i[r][c];
                    Zr[r][c] = Zn_r[r][c];
                    Zi[r][c] = Zn_i[r][c];
                }
        }
        // P0 = C^{-1/2} = A^{-1/2} / sqrt(||C||_F), made exactly Hermitian
        const double sc = 1.0 / sqrt(fn);
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) {
                const double pr = 0.5 * (Zr[r][c] + Zr[c][r]) * sc;
                const double pi = 0.5 * (Zi[r][c] - Zi[c][r]) * sc;
                Ps[r * M + c] = make_double2(pr, pi);
                P0[static_cast<size_t>(f) * M * M + r * M + c] = make_double2(pr, pi);
            }
    }
    __syncthreads();
    // features and their mean over t
    float msum[M];
    for (int m = 0; m < M; ++m) msum[m] = 0.0f;
    float *ff = feat + static_cast<size_t>(f) * M * T;
    for (int t = tid; t < T; t += blockDim.x) {
        for (int m = 0; m < M; ++m) {
            float yr = 0.f, yi = 0.f;
            for (int r = 0; r < M; ++r) {
                const double2 p = Ps[r * M + m];
                const float2 a = xf[static_cast<size_t>(t) * M + r];
                yr += static_cast<float>(p.x) * a.x + static_cast<float>(p.y) * a.y;
                yi += static_cast<float>(p.x) * a.y - static_cast<float>(p.y) * a.x;
            }
            const float v = logf(yr * yr + yi * yi + eps);
            ff[static_cast<size_t>(m) * T + t] = v;
            msum[m] += v;
        }
    }
    for (int m = 0; m < M; ++m) {
        const float v = wave_sum(msum[m]);
        if ((tid & 63) == 0) mred[tid >> 6][m] = v;
    }
    __syncthreads();
    for (int m = 0; m < M; ++m) {
        const float mean = ((mred[0][m] + mred[1][m]) + (mred[2][m] + mred[3][m])) / static_cast<float>(T);
        for (int t = tid; t < T; t += blockDim.x) ff[static_cast<size_t>(m) * T + t] -= mean;
    }
}

// ------------------------------------------------------------------ targets
// From a fit (P, lam, v) and the whitening P0 of each frequency: scale each
// source so that tr R_n = M (R_n = P^{-H} diag(lam_n) P^{-1}, the trace
// normalization of eq:Rerror), target log-powers tv[n][t] = ln(c_n v_tn),
// target log-diagonals tl[n][m] = ln [P0^H (R_n / c_n) P0]_{mm}, c_n = tr R_n / M.
// One thread per frequency; M <= 4.
__global__ void targets_kernel(const double2 *P, const float *lam, const float *v, const double2 *P0, int F,
                               int T, int M, int N, float *tv, float *tl) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    cd A[kFeatMaxM][2 * kFeatMaxM];
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < 2 * M; ++c)
            A[r][c] = c < M ? ld(P[static_cast<size_t>(f) * M * M + r * M + c]) : cmk(c - M == r ? 1.0 : 0.0, 0.0);
    // Gauss-Jordan inverse of P (partial pivoting)
    for (int k = 0; k < M; ++k) {
        int p = k;
        double best = abs2(A[k][k]);
        for (int i = k + 1; i < M; ++i)
            if (abs2(A[i][k]) > best) {
                best = abs2(A[i][k]);
                p = i;
            }
        for (int j = 0; j < 2 * M; ++j) {
            const cd t = A[k][j];
            A[k][j] = A[p][j];
            A[p][j] = t;
        }
        const cd piv = A[k][k];
        for (int j = 0; j < 2 * M; ++j) A[k][j] = cdiv(A[k][j], piv);
        for (int i = 0; i < M; ++i) {
            if (i == k) continue;
            const cd l = A[i][k];
            for (int j = 0; j < 2 * M; ++j) A[i][j] = A[i][j] - l * A[k][j];
        }
    }
    // B = P^{-1} (A[:, M:]); R_n = B^H diag(lam_n) B; G = P0^H R_n P0 diagonal:
    // [P0^H B^H D B P0]_{mm} = sum_k lam_nk |(B P0)_{k m}|^2
    cd BP[kFeatMaxM][kFeatMaxM];
    for (int k = 0; k < M; ++k)
        for (int m = 0; m < M; ++m) {
            cd s = cmk(0.0, 0.0);
            for (int j = 0; j < M; ++j) s = s + A[k][M + j] * ld(P0[static_cast<size_t>(f) * M * M + j * M + m]);
            BP[k][m] = s;
        }
    for (int n = 0; n < N; ++n) {
        // tr R_n = sum_k lam_nk ||B[k,:]||^2
        double tr = 0.0;
        for (int k = 0; k < M; ++k) {
            double rn = 0.0;
            for (int j = 0; j < M; ++j) rn += abs2(A[k][M + j]);
            tr += static_cast<double>(lam[(static_cast<size_t>(f) * N + n) * M + k]) * rn;
        }
        const double cn = tr / M;
        for (int m = 0; m < M; ++m) {
            double g = 0.0;
            for (int k = 0; k < M; ++k) g += static_cast<double>(lam[(static_cast<size_t>(f) * N + n) * M + k]) * abs2(BP[k][m]);
            tl[(static_cast<size_t>(f) * N + n) * M + m] = static_cast<float>(log(g / cn));
        }
        const float lc = static_cast<float>(log(cn));
        for (int t = 0; t < T; ++t)
            tv[(static_cast<size_t>(f) * N + n) * T + t] = logf(v[(static_cast<size_t>(f) * T + t) * N + n]) + lc;
    }
}

// warm-start parameters from the network outputs: v[f][t][n] = exp(lv[f][n][t]),
// lam[f][n][m] = exp(ll[f][n][m]) (clamped to a finite positive range)
__global__ void apply_outputs_kernel(const float *lv, const float *ll, int F, int T, int M, int N, float *v,
                                     float *lam) {
    const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
    const size_t nv = static_cast<size_t>(F) * T * N;
    if (i < nv) {
        const size_t f = i / (static_cast<size_t>(T) * N), r = i % (static_cast<size_t>(T) * N);
        const int t = static_cast<int>(r / N), n = static_cast<int>(r % N);
        const float a = fminf(fmaxf(lv[(f * N + n) * T + t], -60.0f), 60.0f);
        v[i] = expf(a);
    }
    if (i < static_cast<size_t>(F) * N * M) lam[i] = expf(fminf(fmaxf(ll[i], -60.0f), 60.0f));
}

// ------------------------------------------------------------------ launchers
static unsigned grid1(size_t n, int th) {
    size_t g = (n + th - 1) / th;
    return static_cast<unsigned>(g > 65535 ? 65535 : (g < 1 ? 1 : g));
}

hipError_t net_pack_weights(const float *W, int ldw, int Cout, int Cin, int KS, int Kp, int tf, uint16_t *Wb,
                            hipStream_t s) {
    const int rows = tf ? Cin : Cout;
    hipLaunchKernelGGL(pack_weights_kernel, dim3((rows * Kp + 255) / 256), dim3(256), 0, s, W, ldw, Cout, Cin,
                       KS, Kp, tf, Wb);
    return hipGetLastError();
}

hipError_t net_conv_fwd(const float *X, int S, int Cin, int T, const uint16_t *Wb, int Kp, int KS,
                        const float *bias, int Cout, float *Y, int mode, const float *Res, float *Pre,
                        hipStream_t s) {
    if (Cin > kMaxC || Cout > kMaxC || Kp > kMaxKp || Kp % 16 || Kp < Cin * KS) return hipErrorInvalidValue;
    dim3 grid((T + kChunk - 1) / kChunk, S);
    if (KS == 5)
        hipLaunchKernelGGL(conv_fwd_kernel<5>, grid, dim3(256), 0, s, X, Cin, Wb, Kp, bias, Cout, Y, T, mode,
                           Res, Pre);
    else if (KS == 1)
        hipLaunchKernelGGL(conv_fwd_kernel<1>, grid, dim3(256), 0, s, X, Cin, Wb, Kp, bias, Cout, Y, T, mode,
                           Res, Pre);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t net_forward_fused(const float *feat, int S, int M, int T, int C, int L, int N,
                             const uint16_t *const *Wb, const float *const *b, int Kp0, const float *Wv, int ldv,
                             const float *bv, float *lv, float *part, float *pooled, hipStream_t s) {
    if (S < 1 || T < 1 || M < 1 || M > 4 || C < 16 || C > kMaxC || C % 16 || L < 0 || L > kFMaxL || N < 1 ||
        N > kFMaxN || Kp0 % 16 || Kp0 < 5 * M || Kp0 > 32 || 5 * C > kMaxKp || ldv < C)
        return hipErrorInvalidValue;
    FusedNetArgs a;
    a.feat = feat;
    a.lv = lv;
    a.part = part;
    for (int l = 0; l <= kFMaxL; ++l) {
        a.W[l] = l <= L ? Wb[l] : nullptr;
        a.b[l] = l <= L ? b[l] : nullptr;
        if (l <= L && (!a.W[l] || !a.b[l])) return hipErrorInvalidValue;
    }
    a.Wv = Wv;
    a.bv = bv;
    a.S = S;
    a.M = M;
    a.T = T;
    a.C = C;
    a.L = L;
    a.N = N;
    a.Kp0 = Kp0;
    a.ldv = ldv;
    a.ntiles = (T + kFT - 1) / kFT;
    const dim3 grid(a.ntiles, S);
    switch (C) {
        case 16: hipLaunchKernelGGL(net_fused_fwd_kernel<16>, grid, dim3(256), 0, s, a); break;
        case 32: hipLaunchKernelGGL(net_fused_fwd_kernel<32>, grid, dim3(256), 0, s, a); break;
        case 48: hipLaunchKernelGGL(net_fused_fwd_kernel<48>, grid, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(net_fused_fwd_kernel<64>, grid, dim3(256), 0, s, a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pool_tiles_kernel, dim3((S * C + 255) / 256), dim3(256), 0, s, part, S, a.ntiles, C, T,
                       pooled);
    return hipGetLastError();
}

hipError_t net_conv_bwdw(const float *G, int S, int Cout, const float *X, int Cin, int T, int Kp, int KS,
                         float *dW, float *db, hipStream_t s) {
    if (Cin > kMaxC || Cout > kMaxC || Kp > kMaxKp || Kp % 16 || Kp < Cin * KS) return hipErrorInvalidValue;
    dim3 grid((T + kChunk - 1) / kChunk, S);
    if (KS == 5)
        hipLaunchKernelGGL(conv_bwdw_kernel<5>, grid, dim3(256), 0, s, G, Cout, X, Cin, Kp, T, dW, db);
    else if (KS == 1)
        hipLaunchKernelGGL(conv_bwdw_kernel<1>, grid, dim3(256), 0, s, G, Cout, X, Cin, Kp, T, dW, db);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t net_relu_grad(const float *G, const float *Pre, float *out, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(relu_grad_kernel, dim3(grid1(n, 256)), dim3(256), 0, s, G, Pre, out, n);
    return hipGetLastError();
}

hipError_t net_mean_t(const float *H, int SC, int T, float *pooled, hipStream_t s) {
    hipLaunchKernelGGL(mean_t_kernel, dim3(SC), dim3(256), 0, s, H, T, pooled);
    return hipGetLastError();
}

hipError_t net_mean_t_bwd(const float *dpooled, int SC, int T, float *dH, hipStream_t s) {
    const size_t n = static_cast<size_t>(SC) * T;
    hipLaunchKernelGGL(mean_t_bwd_kernel, dim3(grid1(n, 256)), dim3(256), 0, s, dpooled, T, dH, n);
    return hipGetLastError();
}

hipError_t net_linear_fwd(const float *in, int S, int C, const float *Wl, const float *bl, int J, float *out,
                          hipStream_t s) {
    hipLaunchKernelGGL(linear_fwd_kernel, dim3((S * J + 255) / 256), dim3(256), 0, s, in, S, C, Wl, bl, J, out);
    return hipGetLastError();
}

hipError_t net_linear_bwd(const float *in, int S, int C, const float *Wl, int J, const float *g, float *dWl,
                          float *dbl, float *din, hipStream_t s) {
    const int n = max(max(J * C, S * C), J);
    hipLaunchKernelGGL(linear_bwd_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, S, C, Wl, J, g, dWl, dbl,
                       din);
    return hipGetLastError();
}

hipError_t net_pit_loss(const float *lv, const float *tv, const float *ll, const float *tl, int S, int N, int M,
                        int T, float wl, float *loss, int *perm, float *glv, float *gll, hipStream_t s) {
    if (N < 1 || N > kPitMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pit_loss_kernel, dim3(S), dim3(256), 0, s, lv, tv, ll, tl, N, M, T, wl, loss, perm, glv,
                       gll);
    return hipGetLastError();
}

hipError_t net_adamw(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                     float eps, float wd, int step, float gscale, hipStream_t s) {
    const float bc1 = 1.0f - powf(b1, static_cast<float>(step));
    const float bc2 = 1.0f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(adamw_kernel, dim3(grid1(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, wd,
                       bc1, bc2, gscale);
    return hipGetLastError();
}

hipError_t net_features(const float2 *x, int F, int T, int M, float eps, double2 *P0, float *feat,
                        hipStream_t s) {
    switch (M) {
        case 1: hipLaunchKernelGGL(features_kernel<1>, dim3(F), dim3(256), 0, s, x, T, eps, P0, feat); break;
        case 2: hipLaunchKernelGGL(features_kernel<2>, dim3(F), dim3(256), 0, s, x, T, eps, P0, feat); break;
        case 3: hipLaunchKernelGGL(features_kernel<3>, dim3(F), dim3(256), 0, s, x, T, eps, P0, feat); break;
        case 4: hipLaunchKernelGGL(features_kernel<4>, dim3(F), dim3(256), 0, s, x, T, eps, P0, feat); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t net_targets(const double2 *P, const float *lam, const float *v, const double2 *P0, int F, int T, int M,
                       int N, float *tv, float *tl, hipStream_t s) {
    if (M < 1 || M > kFeatMaxM) return hipErrorInvalidValue;
    hipLaunchKernelGGL(targets_kernel, dim3((F + 63) / 64), dim3(64), 0, s, P, lam, v, P0, F, T, M, N, tv, tl);
    return hipGetLastError();
}

hipError_t net_apply_outputs(const float *lv, const float *ll, int F, int T, int M, int N, float *v, float *lam,
                             hipStream_t s) {
    const size_t n = static_cast<size_t>(F) * T * N;
    hipLaunchKernelGGL(apply_outputs_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, lv, ll,
                       F, T, M, N, v, lam);
    return hipGetLastError();
}

}  // namespace ffca
