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
};

namespace {

struct MlpPlan {
    size_t o_params, o_grads, o_am, o_av, o_w1, o_w2, o_w3, o_x, o_h1, o_h2, o_dy, o_dh2, o_dh1, o_y, o_bl, o_loss,
        o_scr, total, nparam, scratch_floats;
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
