// k_closure.hip -- inputs and outputs of the learned vertical-mixing closure.
//
// The closure replaces the vertical diffusivity of the implicit diffusion
// (paper Sec. 5.2) by a per-column network (paper Sec. 3 motivates learned
// parameterizations; Sec. 6 uses a vertical-mixing closure). Two kernels sit
// around the network's products:
//
//  k_features: one thread per column, 64 adjacent columns of a row per
//  workgroup. It builds the column's input vector in LDS, then the workgroup
//  writes its 64 consecutive rows of the (ny nx) x din matrix as one contiguous
//  coalesced run (FP32 or BF16). Order: T (nz), u at centres (nz), v at
//  centres (nz), N^2 = g alpha dT/dz on faces (nz, slot 0 and dry faces 0),
//  centred wind stress (2), restoring flux dz_top (T* - T_top)/tau (1), zero
//  padding. Wet entries are normalised with per-feature mean and standard
//  deviation; dry entries are 0.
//
//  k_kappa_map: network output (log10 diffusivity on each z-face, slot 0 the
//  unused bottom face) to the face field: 10^y clipped to [1e-7, 1] m^2/s on
//  wet interior faces, kappa0 where y is not finite; periodic images too.
#include "ocn_dev.h"

#include <cstdint>

namespace ocn {

constexpr int FW = 64;  // columns per workgroup

__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename R>
__global__ __launch_bounds__(FW) void k_features(const DevState S, int din, const float* __restrict__ norm,
                                                 void* __restrict__ out, int out_bf16) {
    extern __shared__ float sfeat[];  // [FW][din + 1]
    const int t = threadIdx.x, i0 = blockIdx.x * FW, j = blockIdx.y, i = i0 + t;
    const int nx = S.nx, nz = S.nz, ld = din + 1;
    float* my = sfeat + t * ld;
    for (int f = 0; f < din; ++f) my[f] = 0.f;

    if (i < nx) {
        const int K = S.kb[idxk(S, i, j)];
        if (K > 0) {
            auto put = [&](int f, double x) {
                my[f] = norm ? float((x - double(norm[f])) / double(norm[din + f])) : float(x);
            };
            const int kbot = nz - K;
            // east / north neighbours across the domain edge: periodic image or land
            const int ie = (i + 1 < nx) ? i + 1 : (S.periodic_x ? 0 : -1);
            const int jn = (j + 1 < S.ny) ? j + 1 : (S.periodic_y ? 0 : -1);
            const int Kuw = min(K, S.kb[idxk(S, i - 1, j)]);
            const int Kue = ie >= 0 ? min(K, S.kb[idxk(S, ie, j)]) : 0;
            const int Kvs = min(K, S.kb[idxk(S, i, j - 1)]);
            const int Kvn = jn >= 0 ? min(K, S.kb[idxk(S, i, jn)]) : 0;
            const R* T = f3<R>(S.t);
            const R* U = f3<R>(S.u);
            const R* V = f3<R>(S.v);
            double tprev = 0.0;
            for (int k = kbot; k < nz; ++k) {
                const double tk = double(T[idx3(S, i, j, k)]) + S.tref[k];
                put(k, tk);
                const double uw = (k >= nz - Kuw) ? double(U[idx3(S, i, j, k)]) : 0.0;
                const double ue = (k >= nz - Kue) ? double(U[idx3(S, ie, j, k)]) : 0.0;
                put(nz + k, 0.5 * (uw + ue));
                const double vs = (k >= nz - Kvs) ? double(V[idx3(S, i, j, k)]) : 0.0;
                const double vn = (k >= nz - Kvn) ? double(V[idx3(S, i, jn, k)]) : 0.0;
                put(2 * nz + k, 0.5 * (vs + vn));
                if (k > kbot) put(3 * nz + k, S.g * S.alpha * (tk - tprev) / S.dzc[k]);
                tprev = tk;
            }
            const double txe = ie >= 0 ? S.taux[idx2(S, ie, j)] : 0.0;
            const double tyn = jn >= 0 ? S.tauy[idx2(S, i, jn)] : 0.0;
            put(4 * nz, 0.5 * (S.taux[idx2(S, i, j)] + txe));
            put(4 * nz + 1, 0.5 * (S.tauy[idx2(S, i, j)] + tyn));
            // the stored T and T* are both anomalies from the top reference level
            const double q = S.restore_inv > 0.0
                                 ? S.dz[nz - 1] * (S.tstar[idx2(S, i, j)] - double(T[idx3(S, i, j, nz - 1)])) *
                                       S.restore_inv
                                 : 0.0;
            put(4 * nz + 2, q);
        }
    }
    __syncthreads();
    // the workgroup's rows j nx + i0 .. j nx + i0 + nrows - 1 are contiguous
    const int nrows = min(FW, nx - i0);
    const long long base = ((long long)j * nx + i0) * din;
    const int total = nrows * din;
    if (out_bf16) {
        uint16_t* o = static_cast<uint16_t*>(out) + base;
        for (int e = t; e < total; e += FW) o[e] = to_bf16(sfeat[(e / din) * ld + e % din]);
    } else {
        float* o = static_cast<float*>(out) + base;
        for (int e = t; e < total; e += FW) o[e] = sfeat[(e / din) * ld + e % din];
    }
}

__device__ __forceinline__ double face_kappa_of(float y, double kappa0) {
    if (!isfinite(y)) return kappa0;
    return fmin(1.0, fmax(1e-7, exp10(double(y))));
}

template <typename R>
__global__ __launch_bounds__(FW) void k_kappa_map(const DevState S, const float* __restrict__ Y, int ldy,
                                                  double kappa0) {
    const int i = blockIdx.x * FW + threadIdx.x, j = blockIdx.y;
    if (i >= S.nx) return;
    const int nz = S.nz;
    const int kbot = nz - S.kb[idxk(S, i, j)];
    const float* y = Y + ((long long)j * S.nx + i) * ldy;
    R* kw = f3<R>(S.kw);
    for (int k = 0; k < nz; ++k) {
        const R val = (k > kbot) ? R(face_kappa_of(y[k], kappa0)) : R(0);
        kw[idx3(S, i, j, k)] = val;
        for_each_image(S, i, j, S.h, [&](int x, int yy) { kw[idx3(S, x, yy, k)] = val; });
    }
}

// Convective adjustment: from the state at the start of the step, kappa_conv
// on interior wet faces where the water above is colder, hence denser, than
// the water below (N^2 < 0), kappa0 on the other wet faces, 0 on dry ones.
template <typename R>
__global__ __launch_bounds__(FW) void k_convective(const DevState S, double kappa_conv, double kappa0) {
    const int i = blockIdx.x * FW + threadIdx.x, j = blockIdx.y;
    if (i >= S.nx) return;
    const int nz = S.nz;
    const int kbot = nz - S.kb[idxk(S, i, j)];
    const R* T = f3<R>(S.t);
    R* kw = f3<R>(S.kw);
    double below = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double tk = (k >= kbot) ? double(T[idx3(S, i, j, k)]) + S.tref[k] : 0.0;
        const R val = (k > kbot) ? R(tk < below ? kappa_conv : kappa0) : R(0);
        kw[idx3(S, i, j, k)] = val;
        for_each_image(S, i, j, S.h, [&](int x, int y) { kw[idx3(S, x, y, k)] = val; });
        below = tk;
    }
}

template <typename R>
hipError_t launch_convective(const DevState& s, double kappa_conv, double kappa0, hipStream_t st) {
    dim3 grid((s.nx + FW - 1) / FW, s.ny);
    hipLaunchKernelGGL(k_convective<R>, grid, dim3(FW), 0, st, s, kappa_conv, kappa0);
    return hipGetLastError();
}
template hipError_t launch_convective<double>(const DevState&, double, double, hipStream_t);
template hipError_t launch_convective<float>(const DevState&, double, double, hipStream_t);

template <typename R>
__global__ __launch_bounds__(256) void k_fill(R* p, long long n, R v) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e < n) p[e] = v;
}

template <typename R>
hipError_t launch_fill(void* p, long long n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, static_cast<R*>(p), n, R(v));
    return hipGetLastError();
}
template hipError_t launch_fill<double>(void*, long long, double, hipStream_t);
template hipError_t launch_fill<float>(void*, long long, double, hipStream_t);

size_t features_lds(int din) { return (size_t)FW * (din + 1) * sizeof(float); }

template <typename R>
hipError_t launch_features(const DevState& s, int din, const float* norm, void* out, int out_bf16, hipStream_t st) {
    const size_t lds = features_lds(din);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    dim3 grid((s.nx + FW - 1) / FW, s.ny);
    hipLaunchKernelGGL(k_features<R>, grid, dim3(FW), lds, st, s, din, norm, out, out_bf16);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_kappa_map(const DevState& s, const float* Y, int ldy, double kappa0, hipStream_t st) {
    dim3 grid((s.nx + FW - 1) / FW, s.ny);
    hipLaunchKernelGGL(k_kappa_map<R>, grid, dim3(FW), 0, st, s, Y, ldy, kappa0);
    return hipGetLastError();
}

template hipError_t launch_features<double>(const DevState&, int, const float*, void*, int, hipStream_t);
template hipError_t launch_features<float>(const DevState&, int, const float*, void*, int, hipStream_t);
template hipError_t launch_kappa_map<double>(const DevState&, const float*, int, double, hipStream_t);
template hipError_t launch_kappa_map<float>(const DevState&, const float*, int, double, hipStream_t);

}  // namespace ocn
