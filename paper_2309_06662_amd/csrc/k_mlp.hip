// k_mlp.hip -- the per-column closure network on the matrix cores.
//
// A three-layer perceptron (Linear -> ReLU -> Linear -> ReLU -> Linear) maps a
// column's features to its vertical-diffusivity profile. All products are
// BF16 x BF16 with FP32 accumulation on v_mfma_f32_16x16x32_bf16; master
// weights, losses and Adam stay FP32. Paper Sec. 3 motivates learned
// parameterizations of unresolved processes; Sec. 6 names a vertical-mixing
// closure as the one the paper's runs use.
//
// GEMM: C[M x N] = op(A)[M x K] op(B)[K x N] with BF16 A, B (row-major, either
// transposed), a 64 x 64 output tile per 256-thread workgroup, each wave a
// 32 x 32 quarter as 2 x 2 MFMA blocks of 16 x 16, K staged through LDS 32 at
// a time. Epilogues: + bias, ReLU, multiply by a ReLU mask (backward), FP32
// or BF16 output; split-K writes partial tiles that a second kernel sums in a
// fixed order, so every result is deterministic.
#include "ocn_dev.h"

#include <cstdint>

namespace ocn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr int GBM = 64, GBN = 64, GBK = 32, GT = 256;
constexpr int APAD = 8;  // LDS row padding (bf16 elements) against bank conflicts

enum GemmFlags { G_BIAS = 1, G_RELU = 2, G_MASK = 4, G_OUT_BF16 = 8 };

struct GemmArgs {
    const uint16_t* A;  // bf16 bits
    const uint16_t* B;
    const float* bias;        // N, or null
    const uint16_t* mask;     // M x N bf16 activations (ldm): zero where mask <= 0
    void* C;                  // M x N (ldc), FP32 or BF16; for split-K: FP32 partials [split][M][N]
    int M, N, K, lda, ldb, ldc, ldm;
    int transA, transB, flags;
    int ksplit;               // number of K slices (grid.z); > 1 writes partials
};

// Lane layout of v_mfma_f32_16x16x32_bf16: lane l holds row (l % 16) of A and
// column (l % 16) of B, each for k = 8 (l / 16) .. 8 (l / 16) + 7; the 4
// results of a lane are rows 4 (l / 16) + v, v = 0..3, of column l % 16.
__device__ __forceinline__ int frag_row(int lane) { return lane & 15; }
__device__ __forceinline__ int frag_k0(int lane) { return (lane >> 4) * 8; }
__device__ __forceinline__ int acc_row(int lane, int v) { return (lane >> 4) * 4 + v; }
__device__ __forceinline__ int acc_col(int lane) { return lane & 15; }

__global__ __launch_bounds__(GT) void k_gemm_bf16(const GemmArgs g) {
    __shared__ __align__(16) uint16_t As[GBM][GBK + APAD];  // As[m][k]
    __shared__ __align__(16) uint16_t Bs[GBN][GBK + APAD];  // Bs[n][k] (B transposed)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    // K range of this slice
    const int kchunks = (g.K + GBK - 1) / GBK;
    const int per = (kchunks + g.ksplit - 1) / g.ksplit;
    const int kc0 = blockIdx.z * per, kc1 = min(kchunks, kc0 + per);

    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int kc = kc0; kc < kc1; ++kc) {
        const int k0 = kc * GBK;
        // stage op(A) tile 64 x 32 and op(B) tile 32 x 64 (zero outside the matrices)
        for (int e = tid; e < GBM * GBK; e += GT) {
            const int r = e / GBK, kk = e % GBK;
            const int m = m0 + r, k = k0 + kk;
            uint16_t v = 0;
            if (m < g.M && k < g.K) v = g.transA ? g.A[(long long)k * g.lda + m] : g.A[(long long)m * g.lda + k];
            As[r][kk] = v;
        }
        for (int e = tid; e < GBN * GBK; e += GT) {
            const int c = e / GBK, kk = e % GBK;
            const int n = n0 + c, k = k0 + kk;
            uint16_t v = 0;
            if (n < g.N && k < g.K) v = g.transB ? g.B[(long long)n * g.ldb + k] : g.B[(long long)k * g.ldb + n];
            Bs[c][kk] = v;
        }
        __syncthreads();
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const uint16_t* pa = &As[wm + a * 16 + frag_row(lane)][frag_k0(lane)];
            const uint16_t* pb = &Bs[wn + a * 16 + frag_row(lane)][frag_k0(lane)];
            af[a] = *reinterpret_cast<const bf16x8*>(pa);
            bfr[a] = *reinterpret_cast<const bf16x8*>(pb);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }

    // epilogue
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wm + a * 16 + acc_row(lane, v);
                const int n = n0 + wn + b * 16 + acc_col(lane);
                if (m >= g.M || n >= g.N) continue;
                float x = acc[a][b][v];
                if (g.ksplit > 1) {
                    static_cast<float*>(g.C)[((long long)blockIdx.z * g.M + m) * g.N + n] = x;
                    continue;
                }
                if (g.flags & G_BIAS) x += g.bias[n];
                if (g.flags & G_RELU) x = x > 0.f ? x : 0.f;
                if (g.flags & G_MASK) x = bf2f(g.mask[(long long)m * g.ldm + n]) > 0.f ? x : 0.f;
                if (g.flags & G_OUT_BF16) static_cast<uint16_t*>(g.C)[(long long)m * g.ldc + n] = f2bf(x);
                else static_cast<float*>(g.C)[(long long)m * g.ldc + n] = x;
            }
}

// Sum split-K partials in slice order into C (FP32, ldc).
__global__ __launch_bounds__(256) void k_splitk_sum(const float* part, int splits, int M, int N, float* C, int ldc) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)M * N) return;
    const int m = (int)(e / N), n = (int)(e % N);
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[((long long)z * M + m) * N + n];
    C[(long long)m * ldc + n] = s;
}

hipError_t gemm_bf16(const GemmArgs& g0, float* scratch, size_t scratch_floats, hipStream_t st) {
    GemmArgs g = g0;
    dim3 grid((g.N + GBN - 1) / GBN, (g.M + GBM - 1) / GBM, 1);
    int splits = 1;
    if (g0.ksplit > 1) {
        const int kchunks = (g.K + GBK - 1) / GBK;
        splits = min(g0.ksplit, kchunks);
        while (splits > 1 && (size_t)splits * g.M * g.N > scratch_floats) --splits;
    }
    if (splits > 1) {
        float* out = static_cast<float*>(g0.C);
        g.ksplit = splits;
        g.C = scratch;
        grid.z = splits;
        hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(GT), 0, st, g);
        const long long n = (long long)g.M * g.N;
        hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, scratch, splits, g.M,
                           g.N, out, g0.ldc);
    } else {
        g.ksplit = 1;
        hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(GT), 0, st, g);
    }
    return hipGetLastError();
}

// FP32 -> BF16 copy of n values, row by row (rows of `cols` values into a
// destination of leading dimension ld, the padding columns zeroed).
__global__ __launch_bounds__(256) void k_to_bf16(const float* src, int rows, int cols, int lds, uint16_t* dst, int ldd) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)rows * ldd) return;
    const int r = (int)(e / ldd), c = (int)(e % ldd);
    dst[e] = c < cols ? f2bf(src[(long long)r * lds + c]) : (uint16_t)0;
}

// dY = (Y - T) / (n dout) as BF16, and the loss sum (Y - T)^2 / (2 n dout) per block.
__global__ __launch_bounds__(256) void k_mse(const float* Y, const float* T, int n, int dout, float scale,
                                             uint16_t* dY, float* block_loss) {
    __shared__ float red[256];
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (e < (long long)n * dout) {
        const float r = Y[e] - T[e];
        dY[e] = f2bf(r * scale);
        l = 0.5f * r * r * scale;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_loss[blockIdx.x] = red[0];
}

// Column sums of a BF16 matrix (n x cols): bias gradients, fixed order per column.
__global__ __launch_bounds__(256) void k_colsum_bf16(const uint16_t* D, int n, int cols, float* out) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < n; ++r) s += bf2f(D[(long long)r * cols + c]);
    out[c] = s;
}

// One Adam step on FP32 parameters (Kingma and Ba 2015).
__global__ __launch_bounds__(256) void k_adam(float* p, const float* g, float* m, float* v, long long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Sum of per-block losses in block order.
__global__ void k_sum_blocks(const float* part, int nb, float* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += part[b];
    *out = s;
}

// ---------------------------------------------------------------------------
// Fused inference: all three layers of a batch tile in one kernel, with the
// weights resident in LDS for the whole launch.
//
// Each layer is computed transposed, H^T = W^T . A^T: the weights are the
// MFMA A operand (16 output units x 32 inputs from LDS) and the activations
// the B operand (16 batch rows). A lane's accumulators then hold, for batch
// row lane % 16, the output units 16 mb + 4 (lane / 16) + v; two adjacent
// blocks mb = 2c, 2c + 1 give eight units per lane, which become the lane's
// B fragment for input chunk c of the next layer if that layer's weight rows
// list their inputs inside each chunk of 32 in the same order (the packing
// below does so). Activations never leave the registers; a wave carries
// IF_RB blocks of 16 batch rows so each weight fragment read from LDS feeds
// IF_RB products. The grid is one workgroup per CU, striding over tiles.
constexpr int IF_WAVES = 8, IF_T = IF_WAVES * 64, IF_RB = 2;
constexpr int IF_ROWS = IF_WAVES * IF_RB * 16;  // batch rows per tile
constexpr int IF_LDS = 128 * 1024;              // packed weights + biases
constexpr int IF_KC1 = 8, IF_MB = 8, IF_KC = 4;  // max input chunks of layer 1, output blocks, hidden chunks

struct InferShape {
    int din, h1, h2, dout;
    int kc1, mb1, kc2, mb2, kc3, mb3;  // input chunks of 32 and output blocks of 16 of each layer
    int s1, s2, s3;                     // row strides (bf16 elements) of the packed weight matrices
    int o2, o3, ob;                     // element offsets of layer 2, layer 3 and the FP32 biases
    int bytes;                          // size of the packed image, a multiple of 16
};

// Position p inside the packed input range of layer 2 or 3 -> index of the
// previous layer's output unit (the accumulator order described above).
__device__ __forceinline__ int perm_k(int p) {
    const int c = p >> 5, q = p & 31, g = q >> 3, j = q & 7;
    return 32 * c + (j < 4 ? 4 * g + j : 12 + 4 * g + j);
}

// Packed image from the FP32 parameters (W1 din x h1, b1, W2, b2, W3, b3),
// rounded to BF16 as the GEMM path rounds them; padding entries are zero.
__global__ __launch_bounds__(256) void k_pack_infer(const float* __restrict__ params, const InferShape S,
                                                    uint16_t* __restrict__ out) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const float* W1 = params;
    const float* b1 = W1 + (size_t)S.din * S.h1;
    const float* W2 = b1 + S.h1;
    const float* b2 = W2 + (size_t)S.h1 * S.h2;
    const float* W3 = b2 + S.h2;
    const float* b3 = W3 + (size_t)S.h2 * S.dout;
    const int nb = S.h1 + S.h2 + 16 * S.mb3;
    if (e < S.o2) {
        const int m = e / S.s1, p = e % S.s1;
        out[e] = p < S.din ? f2bf(W1[(size_t)p * S.h1 + m]) : (uint16_t)0;
    } else if (e < S.o3) {
        const int m = (e - S.o2) / S.s2, p = (e - S.o2) % S.s2;
        out[e] = p < S.h1 ? f2bf(W2[(size_t)perm_k(p) * S.h2 + m]) : (uint16_t)0;
    } else if (e < S.ob) {
        const int m = (e - S.o3) / S.s3, p = (e - S.o3) % S.s3;
        out[e] = (p < S.h2 && m < S.dout) ? f2bf(W3[(size_t)perm_k(p) * S.dout + m]) : (uint16_t)0;
    } else if (e < S.ob + nb) {
        const int f = e - S.ob;
        float v = 0.f;
        if (f < S.h1) v = b1[f];
        else if (f < S.h1 + S.h2) v = b2[f - S.h1];
        else if (f - S.h1 - S.h2 < S.dout) v = b3[f - S.h1 - S.h2];
        reinterpret_cast<float*>(out + S.ob)[f] = v;
    }
}

__device__ __forceinline__ __bf16 relu_bf(float x) { return static_cast<__bf16>(x > 0.f ? x : 0.f); }

__global__ __launch_bounds__(IF_T) void k_mlp_infer(const uint16_t* __restrict__ X, int rows, int ldx,
                                                    const uint16_t* __restrict__ packed, const InferShape S,
                                                    float* __restrict__ Y, int ldy) {
    __shared__ __align__(16) uint16_t W[IF_LDS / 2];
    {
        const uint4* src = reinterpret_cast<const uint4*>(packed);
        uint4* dst = reinterpret_cast<uint4*>(W);
        for (int e = threadIdx.x; e < S.bytes / 16; e += IF_T) dst[e] = src[e];
    }
    __syncthreads();
    const float* bias = reinterpret_cast<const float*>(W + S.ob);
    const uint16_t* W2 = W + S.o2;
    const uint16_t* W3 = W + S.o3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int ntiles = (rows + IF_ROWS - 1) / IF_ROWS;
    const bf16x8 zero8 = {};
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};

    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int row0 = t * IF_ROWS + wave * (IF_RB * 16);
        // layer 1 inputs: lane holds X[row][32 c + 8 g .. + 7] of its batch row in each block
        bf16x8 xb[IF_RB][IF_KC1];
#pragma unroll
        for (int rb = 0; rb < IF_RB; ++rb) {
            const int row = row0 + rb * 16 + r16;
#pragma unroll
            for (int c = 0; c < IF_KC1; ++c) {
                const int k = 32 * c + 8 * g;
                xb[rb][c] = (c < S.kc1 && row < rows && k < S.din)
                                ? *reinterpret_cast<const bf16x8*>(X + (size_t)row * ldx + k)
                                : zero8;
            }
        }
        f32x4 acc[IF_MB][IF_RB];
#pragma unroll
        for (int mb = 0; mb < IF_MB; ++mb)
#pragma unroll
            for (int rb = 0; rb < IF_RB; ++rb) acc[mb][rb] = zero4;
#pragma unroll
        for (int c = 0; c < IF_KC1; ++c) {
            if (c >= S.kc1) break;
#pragma unroll
            for (int mb = 0; mb < IF_MB; ++mb) {
                if (mb >= S.mb1) break;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(W + (mb * 16 + r16) * S.s1 + 32 * c + 8 * g);
#pragma unroll
                for (int rb = 0; rb < IF_RB; ++rb)
                    acc[mb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, xb[rb][c], acc[mb][rb], 0, 0, 0);
            }
        }
        // hidden layers: bias, ReLU, BF16, straight into the next layer's B fragments
        bf16x8 hb[IF_KC][IF_RB];
        int boff = 0;
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            const int kc = layer == 0 ? S.kc2 : S.kc3;
            const int mb_next = layer == 0 ? S.mb2 : S.mb3;
            const int s = layer == 0 ? S.s2 : S.s3;
            const uint16_t* Wn = layer == 0 ? W2 : W3;
#pragma unroll
            for (int c = 0; c < IF_KC; ++c) {
#pragma unroll
                for (int rb = 0; rb < IF_RB; ++rb) {
                    bf16x8 h = zero8;
                    if (c < kc) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            h[j] = relu_bf(acc[2 * c][rb][j] + bias[boff + 32 * c + 4 * g + j]);
                            h[4 + j] = relu_bf(acc[2 * c + 1][rb][j] + bias[boff + 32 * c + 16 + 4 * g + j]);
                        }
                    }
                    hb[c][rb] = h;
                }
            }
            boff += layer == 0 ? S.h1 : S.h2;
#pragma unroll
            for (int mb = 0; mb < IF_MB; ++mb)
#pragma unroll
                for (int rb = 0; rb < IF_RB; ++rb) acc[mb][rb] = zero4;
#pragma unroll
            for (int c = 0; c < IF_KC; ++c) {
                if (c >= kc) break;
#pragma unroll
                for (int mb = 0; mb < IF_MB; ++mb) {
                    if (mb >= mb_next) break;
                    const bf16x8 a = *reinterpret_cast<const bf16x8*>(Wn + (mb * 16 + r16) * s + 32 * c + 8 * g);
#pragma unroll
                    for (int rb = 0; rb < IF_RB; ++rb)
                        acc[mb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[c][rb], acc[mb][rb], 0, 0, 0);
                }
            }
        }
        // outputs: lane holds units 16 mb + 4 g + v of its batch row
#pragma unroll
        for (int rb = 0; rb < IF_RB; ++rb) {
            const int row = row0 + rb * 16 + r16;
            if (row >= rows) continue;
#pragma unroll
            for (int mb = 0; mb < IF_MB; ++mb) {
                if (mb >= S.mb3) break;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int o = 16 * mb + 4 * g + v;
                    if (o < S.dout) Y[(size_t)row * ldy + o] = acc[mb][rb][v] + bias[boff + o];
                }
            }
        }
    }
}

// Layout of the packed image for a network shape; false if the fused kernel
// does not take it (then inference runs layer by layer on the GEMM kernel).
bool infer_shape(int din, int h1, int h2, int dout, InferShape* out) {
    InferShape S{};
    S.din = din; S.h1 = h1; S.h2 = h2; S.dout = dout;
    if (din % 8 || h1 % 32 || h2 % 32 || din > 32 * IF_KC1 || h1 > 32 * IF_KC || h2 > 32 * IF_KC || dout > 16 * IF_MB)
        return false;
    S.kc1 = (din + 31) / 32; S.mb1 = h1 / 16;
    S.kc2 = h1 / 32; S.mb2 = h2 / 16;
    S.kc3 = h2 / 32; S.mb3 = (dout + 15) / 16;
    // strides of 8 mod 16 elements put the 16 rows of a fragment read on distinct banks
    S.s1 = 32 * S.kc1 + 8; S.s2 = h1 + 8; S.s3 = h2 + 8;
    S.o2 = h1 * S.s1;
    S.o3 = S.o2 + h2 * S.s2;
    S.ob = (S.o3 + 16 * S.mb3 * S.s3 + 7) / 8 * 8;
    S.bytes = (2 * S.ob + 4 * (h1 + h2 + 16 * S.mb3) + 15) / 16 * 16;
    if (S.bytes > IF_LDS) return false;
    *out = S;
    return true;
}

}  // namespace ocn

// ---------------------------------------------------------------------------
// Host side: one network with its buffers in a caller arena.

#include "ocn.h"

#include <cmath>
#include <string>
#include <vector>

namespace ocn {
int set_error(int code, const char* msg);
}

struct ocn_mlp {
    int din, h1, h2, dout, max_batch;
    hipStream_t st;
    size_t nparam;
    float *params, *grads, *am, *av;            // FP32 master weights, gradients, Adam moments
    uint16_t *W1b, *W2b, *W3b;                   // BF16 copies
    uint16_t *Xb, *H1b, *H2b, *dYb, *dH2b, *dH1b;
    float *Y, *block_loss, *loss, *scratch;
    size_t scratch_floats;
    int t;                                       // Adam step count
    bool fused;                                  // shape taken by the fused inference kernel
    ocn::InferShape is;                          // its packed-weight layout
    uint16_t* packed;                            // packed BF16 weights + FP32 biases (is.bytes)
    int cus;                                     // compute units of the device (fused grid size)
};

namespace {

struct MlpPlan {
    size_t o_params, o_grads, o_am, o_av, o_w1, o_w2, o_w3, o_x, o_h1, o_h2, o_dy, o_dh2, o_dh1, o_y, o_bl, o_loss,
        o_scr, o_pk, total, nparam, scratch_floats;
    bool fused;
    ocn::InferShape is;
};

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

MlpPlan mlp_plan(int din, int h1, int h2, int dout, int nb) {
    MlpPlan P{};
    P.nparam = (size_t)din * h1 + h1 + (size_t)h1 * h2 + h2 + (size_t)h2 * dout + dout;
    P.scratch_floats = (size_t)16 * (size_t)std::max({din * h1, h1 * h2, h2 * dout});
    size_t off = 0;
    auto add = [&](size_t bytes) { size_t o = off; off = up256(off + bytes); return o; };
    P.o_params = add(P.nparam * 4);
    P.o_grads = add(P.nparam * 4);
    P.o_am = add(P.nparam * 4);
    P.o_av = add(P.nparam * 4);
    P.o_w1 = add((size_t)din * h1 * 2);
    P.o_w2 = add((size_t)h1 * h2 * 2);
    P.o_w3 = add((size_t)h2 * dout * 2);
    P.o_x = add((size_t)nb * din * 2);
    P.o_h1 = add((size_t)nb * h1 * 2);
    P.o_h2 = add((size_t)nb * h2 * 2);
    P.o_dy = add((size_t)nb * dout * 2);
    P.o_dh2 = add((size_t)nb * h2 * 2);
    P.o_dh1 = add((size_t)nb * h1 * 2);
    P.o_y = add((size_t)nb * dout * 4);
    P.o_bl = add((size_t)((nb * dout + 255) / 256 + 1) * 4);
    P.o_loss = add(4);
    P.o_scr = add(P.scratch_floats * 4);
    P.fused = ocn::infer_shape(din, h1, h2, dout, &P.is);
    P.o_pk = add(P.fused ? (size_t)P.is.bytes : 0);
    P.total = off;
    return P;
}

#define MLPCHK(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return ocn::set_error(OCN_E_DEVICE, hipGetErrorString(e_));            \
    } while (0)

int refresh_bf16(ocn_mlp* n) {
    const float* W1 = n->params;
    const float* W2 = W1 + (size_t)n->din * n->h1 + n->h1;
    const float* W3 = W2 + (size_t)n->h1 * n->h2 + n->h2;
    auto conv = [&](const float* src, int rows, int cols, uint16_t* dst) {
        const long long tot = (long long)rows * cols;
        hipLaunchKernelGGL(ocn::k_to_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, n->st, src, rows, cols,
                           cols, dst, cols);
    };
    conv(W1, n->din, n->h1, n->W1b);
    conv(W2, n->h1, n->h2, n->W2b);
    conv(W3, n->h2, n->dout, n->W3b);
    if (n->fused) {
        const int tot = n->is.ob + n->is.h1 + n->is.h2 + 16 * n->is.mb3;
        hipLaunchKernelGGL(ocn::k_pack_infer, dim3((tot + 255) / 256), dim3(256), 0, n->st, n->params, n->is,
                           n->packed);
    }
    MLPCHK(hipGetLastError());
    return OCN_OK;
}

ocn::GemmArgs gemm(const uint16_t* A, const uint16_t* B, void* C, int M, int N, int K, int lda, int ldb, int ldc,
                   int ta, int tb, int flags, const float* bias, const uint16_t* mask, int ldm, int ksplit) {
    ocn::GemmArgs g{};
    g.A = A; g.B = B; g.C = C; g.M = M; g.N = N; g.K = K; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.transA = ta; g.transB = tb; g.flags = flags; g.bias = bias; g.mask = mask; g.ldm = ldm; g.ksplit = ksplit;
    return g;
}

int forward(ocn_mlp* n, const float* x, int rows) {
    const float* b1 = n->params + (size_t)n->din * n->h1;
    const float* b2 = b1 + n->h1 + (size_t)n->h1 * n->h2;
    const float* b3 = b2 + n->h2 + (size_t)n->h2 * n->dout;
    const long long tot = (long long)rows * n->din;
    hipLaunchKernelGGL(ocn::k_to_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, n->st, x, rows, n->din,
                       n->din, n->Xb, n->din);
    using namespace ocn;
    MLPCHK(gemm_bf16(gemm(n->Xb, n->W1b, n->H1b, rows, n->h1, n->din, n->din, n->h1, n->h1, 0, 0,
                          G_BIAS | G_RELU | G_OUT_BF16, b1, nullptr, 0, 1), n->scratch, n->scratch_floats, n->st));
    MLPCHK(gemm_bf16(gemm(n->H1b, n->W2b, n->H2b, rows, n->h2, n->h1, n->h1, n->h2, n->h2, 0, 0,
                          G_BIAS | G_RELU | G_OUT_BF16, b2, nullptr, 0, 1), n->scratch, n->scratch_floats, n->st));
    MLPCHK(gemm_bf16(gemm(n->H2b, n->W3b, n->Y, rows, n->dout, n->h2, n->h2, n->dout, n->dout, 0, 0, G_BIAS, b3,
                          nullptr, 0, 1), n->scratch, n->scratch_floats, n->st));
    return OCN_OK;
}

int backward(ocn_mlp* n, const float* t, int rows) {
    using namespace ocn;
    float* gW1 = n->grads;
    float* gb1 = gW1 + (size_t)n->din * n->h1;
    float* gW2 = gb1 + n->h1;
    float* gb2 = gW2 + (size_t)n->h1 * n->h2;
    float* gW3 = gb2 + n->h2;
    float* gb3 = gW3 + (size_t)n->h2 * n->dout;
    const long long ny = (long long)rows * n->dout;
    const int nb = (int)((ny + 255) / 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, n->st, n->Y, t, rows, n->dout, 1.f / (float)ny, n->dYb,
                       n->block_loss);
    hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(64), 0, n->st, n->block_loss, nb, n->loss);
    const int ks = std::max(1, std::min(16, rows / 512));
    // layer 3
    MLPCHK(gemm_bf16(gemm(n->H2b, n->dYb, gW3, n->h2, n->dout, rows, n->h2, n->dout, n->dout, 1, 0, 0, nullptr,
                          nullptr, 0, ks), n->scratch, n->scratch_floats, n->st));
    hipLaunchKernelGGL(k_colsum_bf16, dim3((n->dout + 255) / 256), dim3(256), 0, n->st, n->dYb, rows, n->dout, gb3);
    MLPCHK(gemm_bf16(gemm(n->dYb, n->W3b, n->dH2b, rows, n->h2, n->dout, n->dout, n->dout, n->h2, 0, 1,
                          G_MASK | G_OUT_BF16, nullptr, n->H2b, n->h2, 1), n->scratch, n->scratch_floats, n->st));
    // layer 2
    MLPCHK(gemm_bf16(gemm(n->H1b, n->dH2b, gW2, n->h1, n->h2, rows, n->h1, n->h2, n->h2, 1, 0, 0, nullptr, nullptr,
                          0, ks), n->scratch, n->scratch_floats, n->st));
    hipLaunchKernelGGL(k_colsum_bf16, dim3((n->h2 + 255) / 256), dim3(256), 0, n->st, n->dH2b, rows, n->h2, gb2);
    MLPCHK(gemm_bf16(gemm(n->dH2b, n->W2b, n->dH1b, rows, n->h1, n->h2, n->h2, n->h2, n->h1, 0, 1,
                          G_MASK | G_OUT_BF16, nullptr, n->H1b, n->h1, 1), n->scratch, n->scratch_floats, n->st));
    // layer 1
    MLPCHK(gemm_bf16(gemm(n->Xb, n->dH1b, gW1, n->din, n->h1, rows, n->din, n->h1, n->h1, 1, 0, 0, nullptr, nullptr,
                          0, ks), n->scratch, n->scratch_floats, n->st));
    hipLaunchKernelGGL(k_colsum_bf16, dim3((n->h1 + 255) / 256), dim3(256), 0, n->st, n->dH1b, rows, n->h1, gb1);
    MLPCHK(hipGetLastError());
    return OCN_OK;
}

}  // namespace

namespace ocn {

void mlp_shape(const ::ocn_mlp* n, int* din, int* h1, int* h2, int* dout) {
    *din = n->din; *h1 = n->h1; *h2 = n->h2; *dout = n->dout;
}

// Forward pass of the network over rows already in BF16, on the caller's
// stream and buffers (no split-K, so no scratch is needed).
hipError_t mlp_infer(const ::ocn_mlp* n, const uint16_t* Xb, int rows, uint16_t* H1b, uint16_t* H2b, float* Y,
                     hipStream_t st) {
    if (n->fused) {
        const int tiles = (rows + IF_ROWS - 1) / IF_ROWS;
        hipLaunchKernelGGL(k_mlp_infer, dim3(std::max(1, std::min(tiles, n->cus))), dim3(IF_T), 0, st, Xb, rows,
                           n->din, n->packed, n->is, Y, n->dout);
        return hipGetLastError();
    }
    const float* b1 = n->params + (size_t)n->din * n->h1;
    const float* b2 = b1 + n->h1 + (size_t)n->h1 * n->h2;
    const float* b3 = b2 + n->h2 + (size_t)n->h2 * n->dout;
    hipError_t e = gemm_bf16(gemm(Xb, n->W1b, H1b, rows, n->h1, n->din, n->din, n->h1, n->h1, 0, 0,
                                  G_BIAS | G_RELU | G_OUT_BF16, b1, nullptr, 0, 1), nullptr, 0, st);
    if (e != hipSuccess) return e;
    e = gemm_bf16(gemm(H1b, n->W2b, H2b, rows, n->h2, n->h1, n->h1, n->h2, n->h2, 0, 0, G_BIAS | G_RELU | G_OUT_BF16,
                       b2, nullptr, 0, 1), nullptr, 0, st);
    if (e != hipSuccess) return e;
    return gemm_bf16(gemm(H2b, n->W3b, Y, rows, n->dout, n->h2, n->h2, n->dout, n->dout, 0, 0, G_BIAS, b3, nullptr,
                          0, 1), nullptr, 0, st);
}

}  // namespace ocn

extern "C" {

int ocn_mlp_arena_bytes(int32_t din, int32_t h1, int32_t h2, int32_t dout, int32_t max_batch, size_t* bytes) {
    if (din < 1 || h1 < 1 || h2 < 1 || dout < 1 || max_batch < 1 || !bytes)
        return ocn::set_error(OCN_E_INVALID, "sizes must be >= 1 and bytes non-NULL");
    *bytes = mlp_plan(din, h1, h2, dout, max_batch).total;
    return OCN_OK;
}

int ocn_mlp_init(int32_t din, int32_t h1, int32_t h2, int32_t dout, int32_t max_batch, void* arena, size_t bytes,
                 void* stream, ocn_mlp** out) {
    size_t need = 0;
    int rc = ocn_mlp_arena_bytes(din, h1, h2, dout, max_batch, &need);
    if (rc) return rc;
    if (!arena || !out) return ocn::set_error(OCN_E_INVALID, "arena and out must not be NULL");
    if (reinterpret_cast<uintptr_t>(arena) % 256) return ocn::set_error(OCN_E_INVALID, "arena must be 256-byte aligned");
    if (bytes < need) return ocn::set_error(OCN_E_NOMEM, "arena smaller than ocn_mlp_arena_bytes");
    const MlpPlan P = mlp_plan(din, h1, h2, dout, max_batch);
    unsigned char* A = static_cast<unsigned char*>(arena);
    ocn_mlp* n = new ocn_mlp();
    n->din = din; n->h1 = h1; n->h2 = h2; n->dout = dout; n->max_batch = max_batch;
    n->st = static_cast<hipStream_t>(stream);
    n->nparam = P.nparam;
    n->params = reinterpret_cast<float*>(A + P.o_params);
    n->grads = reinterpret_cast<float*>(A + P.o_grads);
    n->am = reinterpret_cast<float*>(A + P.o_am);
    n->av = reinterpret_cast<float*>(A + P.o_av);
    n->W1b = reinterpret_cast<uint16_t*>(A + P.o_w1);
    n->W2b = reinterpret_cast<uint16_t*>(A + P.o_w2);
    n->W3b = reinterpret_cast<uint16_t*>(A + P.o_w3);
    n->Xb = reinterpret_cast<uint16_t*>(A + P.o_x);
    n->H1b = reinterpret_cast<uint16_t*>(A + P.o_h1);
    n->H2b = reinterpret_cast<uint16_t*>(A + P.o_h2);
    n->dYb = reinterpret_cast<uint16_t*>(A + P.o_dy);
    n->dH2b = reinterpret_cast<uint16_t*>(A + P.o_dh2);
    n->dH1b = reinterpret_cast<uint16_t*>(A + P.o_dh1);
    n->Y = reinterpret_cast<float*>(A + P.o_y);
    n->block_loss = reinterpret_cast<float*>(A + P.o_bl);
    n->loss = reinterpret_cast<float*>(A + P.o_loss);
    n->scratch = reinterpret_cast<float*>(A + P.o_scr);
    n->scratch_floats = P.scratch_floats;
    n->t = 0;
    n->fused = P.fused;
    n->is = P.is;
    n->packed = reinterpret_cast<uint16_t*>(A + P.o_pk);
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
            delete n;
            return ocn::set_error(OCN_E_DEVICE, "cannot query the compute-unit count");
        }
        n->cus = cus;
    }
    hipError_t e = hipMemsetAsync(arena, 0, P.total, n->st);
    if (e == hipSuccess) e = hipStreamSynchronize(n->st);
    if (e != hipSuccess) {
        delete n;
        return ocn::set_error(OCN_E_DEVICE, hipGetErrorString(e));
    }
    *out = n;
    return OCN_OK;
}

void ocn_mlp_destroy(ocn_mlp* n) {
    if (n) {
        (void)hipStreamSynchronize(n->st);
        delete n;
    }
}

int ocn_mlp_param_count(const ocn_mlp* n, size_t* count) {
    if (!n || !count) return ocn::set_error(OCN_E_INVALID, "NULL argument");
    *count = n->nparam;
    return OCN_OK;
}

int ocn_mlp_set_params(ocn_mlp* n, const float* host, size_t count) {
    if (!n || !host || count != n->nparam) return ocn::set_error(OCN_E_INVALID, "bad parameter buffer");
    MLPCHK(hipMemcpyAsync(n->params, host, count * 4, hipMemcpyHostToDevice, n->st));
    MLPCHK(hipMemsetAsync(n->am, 0, count * 4, n->st));
    MLPCHK(hipMemsetAsync(n->av, 0, count * 4, n->st));
    n->t = 0;
    int rc = refresh_bf16(n);
    if (rc) return rc;
    MLPCHK(hipStreamSynchronize(n->st));
    return OCN_OK;
}

int ocn_mlp_get_params(ocn_mlp* n, float* host, size_t count) {
    if (!n || !host || count != n->nparam) return ocn::set_error(OCN_E_INVALID, "bad parameter buffer");
    MLPCHK(hipMemcpyAsync(host, n->params, count * 4, hipMemcpyDeviceToHost, n->st));
    MLPCHK(hipStreamSynchronize(n->st));
    return OCN_OK;
}

int ocn_mlp_forward(ocn_mlp* n, const float* x_dev, int32_t rows, float* y_dev) {
    if (!n || !x_dev || !y_dev || rows < 1 || rows > n->max_batch) return ocn::set_error(OCN_E_INVALID, "bad arguments");
    if (n->fused) {
        const long long tot = (long long)rows * n->din;
        hipLaunchKernelGGL(ocn::k_to_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, n->st, x_dev, rows,
                           n->din, n->din, n->Xb, n->din);
        MLPCHK(ocn::mlp_infer(n, n->Xb, rows, n->H1b, n->H2b, y_dev, n->st));
        return OCN_OK;
    }
    int rc = forward(n, x_dev, rows);
    if (rc) return rc;
    MLPCHK(hipMemcpyAsync(y_dev, n->Y, (size_t)rows * n->dout * 4, hipMemcpyDeviceToDevice, n->st));
    return OCN_OK;
}

int ocn_mlp_gradients(ocn_mlp* n, const float* x_dev, const float* t_dev, int32_t rows, float* grads_host,
                      size_t count, float* loss_host) {
    if (!n || !x_dev || !t_dev || rows < 1 || rows > n->max_batch || (grads_host && count != n->nparam))
        return ocn::set_error(OCN_E_INVALID, "bad arguments");
    int rc = forward(n, x_dev, rows);
    if (rc) return rc;
    if ((rc = backward(n, t_dev, rows))) return rc;
    if (grads_host) MLPCHK(hipMemcpyAsync(grads_host, n->grads, count * 4, hipMemcpyDeviceToHost, n->st));
    if (loss_host) MLPCHK(hipMemcpyAsync(loss_host, n->loss, 4, hipMemcpyDeviceToHost, n->st));
    MLPCHK(hipStreamSynchronize(n->st));
    return OCN_OK;
}

int ocn_mlp_train_step(ocn_mlp* n, const float* x_dev, const float* t_dev, int32_t rows, float lr, float* loss_host) {
    if (!n || !x_dev || !t_dev || rows < 1 || rows > n->max_batch || !(lr > 0.f))
        return ocn::set_error(OCN_E_INVALID, "bad arguments");
    int rc = forward(n, x_dev, rows);
    if (rc) return rc;
    if ((rc = backward(n, t_dev, rows))) return rc;
    n->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->t), c2 = 1.f - std::pow(b2, (float)n->t);
    hipLaunchKernelGGL(ocn::k_adam, dim3((unsigned)((n->nparam + 255) / 256)), dim3(256), 0, n->st, n->params, n->grads,
                       n->am, n->av, (long long)n->nparam, lr, b1, b2, 1e-8f, c1, c2);
    if ((rc = refresh_bf16(n))) return rc;
    if (loss_host) {
        MLPCHK(hipMemcpyAsync(loss_host, n->loss, 4, hipMemcpyDeviceToHost, n->st));
        MLPCHK(hipStreamSynchronize(n->st));
    }
    return OCN_OK;
}

}  // extern "C"
