// k_closure.hip -- inputs and outputs of the learned vertical-mixing closure.
//
// The closure replaces the vertical diffusivity of the implicit diffusion
// (paper Sec. 5.2) by a per-column network (paper Sec. 3 motivates learned
// parameterizations; Sec. 6 uses a vertical-mixing closure). Two kernels sit
// around the network's products:
//
//  k_features: 64 adjacent columns of a row per workgroup, four threads per
//  column taking every fourth level. They build the columns' input vectors
//  in LDS, then the workgroup writes its 64 consecutive rows of the
//  (ny nx) x din matrix as one contiguous coalesced run (FP32 or BF16). Order: T (nz), u at centres (nz), v at
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

constexpr int FG = 4;   // level groups per workgroup: thread (t, g) takes levels g, g + FG, ...
constexpr int FCH = 4;  // levels whose loads a thread issues together

// Stores a workgroup's rows (contiguous in the output) from the LDS tile
// [FW][ld]: whole rows of n values are written by consecutive threads.
template <typename O>
__device__ __forceinline__ void store_rows(const O* tile, int ld, int nrows, int n, O* out) {
    constexpr int NT = FW * FG;
    const int tid = threadIdx.y * FW + threadIdx.x;
    if (n >= NT) {
        for (int r = 0; r < nrows; ++r)
            for (int f = tid; f < n; f += NT) out[(long long)r * n + f] = tile[r * ld + f];
    } else {
        const int rpi = NT / n, r0 = tid / n, f = tid - r0 * n;
        if (r0 < rpi)
            for (int r = r0; r < nrows; r += rpi) out[(long long)r * n + f] = tile[r * ld + f];
    }
}

__device__ __forceinline__ void put_feature(float* tile, int f, float x) { tile[f] = x; }
__device__ __forceinline__ void put_feature(uint16_t* tile, int f, float x) { tile[f] = to_bf16(x); }

// O = float (FP32 rows) or uint16_t (BF16 rows). The row tile is staged in
// the output type, so BF16 rows need half the LDS.
template <typename R, typename O>
__global__ __launch_bounds__(FW * FG) void k_features(const DevState S, int din, const float* __restrict__ norm,
                                                      O* __restrict__ out) {
    extern __shared__ __align__(16) unsigned char feat_smem[];
    O* tile = reinterpret_cast<O*>(feat_smem);
    const int ld = din + (sizeof(O) == 4 ? 1 : 2);
    // a wave is one level group (the block is 64 wide), so g is uniform across it
    const int t = threadIdx.x, g = __builtin_amdgcn_readfirstlane(threadIdx.y), i0 = blockIdx.x * FW, j = blockIdx.y;
    const int i = i0 + t;
    const int nx = S.nx, nz = S.nz;
    O* my = tile + t * ld;

    if (i < nx) {
        const int K = S.kb[idxk(S, i, j)];
        const int kbot = nz - K;
        // normalisation in the state's precision: FP64 states divide in FP64;
        // FP32 states take (x - mean) times the FP32 reciprocal deviation
        auto put = [&](int f, double x) {
            float v;
            if constexpr (sizeof(R) == 8) {
                v = norm ? float((x - double(norm[f])) / double(norm[din + f])) : float(x);
            } else {
                const float xf = float(x);
                v = norm ? (xf - norm[f]) * __builtin_amdgcn_rcpf(norm[din + f]) : xf;
            }
            put_feature(my, f, v);
        };
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
        // the loads of FCH of this thread's levels are issued together
        // (addresses clamped to valid points, masks applied afterwards)
        const int iec = ie >= 0 ? ie : i, jnc = jn >= 0 ? jn : j;
        for (int m0 = 0; g + FG * m0 < nz; m0 += FCH) {
            R vT[FCH], vTb[FCH], vUw[FCH], vUe[FCH], vVs[FCH], vVn[FCH];
#pragma unroll
            for (int m = 0; m < FCH; ++m) {
                const int k = g + FG * (m0 + m);
                if (k < nz) {
                    vT[m] = T[idx3(S, i, j, k)];
                    vTb[m] = T[idx3(S, i, j, max(k - 1, 0))];
                    vUw[m] = U[idx3(S, i, j, k)];
                    vUe[m] = U[idx3(S, iec, j, k)];
                    vVs[m] = V[idx3(S, i, j, k)];
                    vVn[m] = V[idx3(S, i, jnc, k)];
                }
            }
#pragma unroll
            for (int m = 0; m < FCH; ++m) {
                const int k = g + FG * (m0 + m);
                if (k >= nz) break;
                if (k < kbot) {
                    put_feature(my, k, 0.f);
                    put_feature(my, nz + k, 0.f);
                    put_feature(my, 2 * nz + k, 0.f);
                    put_feature(my, 3 * nz + k, 0.f);
                    continue;
                }
                const double tk = double(vT[m]) + S.tref[k];
                put(k, tk);
                const double uw = (k >= nz - Kuw) ? double(vUw[m]) : 0.0;
                const double ue = (k >= nz - Kue) ? double(vUe[m]) : 0.0;
                put(nz + k, 0.5 * (uw + ue));
                const double vs = (k >= nz - Kvs) ? double(vVs[m]) : 0.0;
                const double vn = (k >= nz - Kvn) ? double(vVn[m]) : 0.0;
                put(2 * nz + k, 0.5 * (vs + vn));
                if (k > kbot) {
                    const double tb = double(vTb[m]) + S.tref[k - 1];
                    put(3 * nz + k, S.g * S.alpha * (tk - tb) / S.dzc[k]);
                } else {
                    put_feature(my, 3 * nz + k, 0.f);
                }
            }
        }
        if (g == 0) {
            if (K > 0) {
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
            } else {
                for (int f = 4 * nz; f < 4 * nz + 3; ++f) put_feature(my, f, 0.f);
            }
            for (int f = 4 * nz + 3; f < din; ++f) put_feature(my, f, 0.f);
        }
    }
    __syncthreads();
    // the workgroup's rows j nx + i0 .. j nx + i0 + nrows - 1 are contiguous
    store_rows(tile, ld, min(FW, nx - i0), din, out + ((long long)j * nx + i0) * din);
}

// 10^y clipped to [1e-7, 1], kappa0 where y is not finite; in the state's
// precision (FP32 states take the FP32 exp10).
template <typename R> __device__ __forceinline__ R face_kappa_of(float y, double kappa0);
template <> __device__ __forceinline__ double face_kappa_of<double>(float y, double kappa0) {
    if (!isfinite(y)) return kappa0;
    return fmin(1.0, fmax(1e-7, exp10(double(y))));
}
template <> __device__ __forceinline__ float face_kappa_of<float>(float y, double kappa0) {
    if (!isfinite(y)) return float(kappa0);
    return fminf(1.0f, fmaxf(1e-7f, exp10f(y)));
}

// The workgroup's 64 output rows are read into LDS in row order (coalesced),
// then each thread writes its column's faces level by level (coalesced
// across the columns).
template <typename R>
__global__ __launch_bounds__(FW * FG) void k_kappa_map(const DevState S, const float* __restrict__ Y, int ldy,
                                                       double kappa0) {
    extern __shared__ __align__(16) unsigned char kap_smem[];
    float* sy = reinterpret_cast<float*>(kap_smem);  // [FW][nz + 1]
    const int nz = S.nz, ld = nz + 1;
    const int t = threadIdx.x, g = __builtin_amdgcn_readfirstlane(threadIdx.y), i0 = blockIdx.x * FW, j = blockIdx.y;
    const int i = i0 + t;
    const int nrows = min(FW, S.nx - i0);
    {
        constexpr int NT = FW * FG;
        const int tid = g * FW + t;
        const float* src = Y + ((long long)j * S.nx + i0) * ldy;
        for (int e = tid; e < nrows * ld; e += NT) {
            const int r = e / ld, k = e - r * ld;
            if (k < nz) sy[e] = src[(long long)r * ldy + k];
        }
    }
    __syncthreads();
    if (i >= S.nx) return;
    const int kbot = nz - S.kb[idxk(S, i, j)];
    R* kw = f3<R>(S.kw);
    for (int k = g; k < nz; k += FG) {
        const R val = (k > kbot) ? face_kappa_of<R>(sy[t * ld + k], kappa0) : R(0);
        kw[idx3(S, i, j, k)] = val;
        for_each_image(S, i, j, S.h, [&](int x, int yy) { kw[idx3(S, x, yy, k)] = val; });
    }
}

// Buoyancy of water (T, S) at depth z under the quadratic equation of state
// (Roquet et al. 2015, the simplified form): rho' = -a0 (1 + lambda1 Ta/2 +
// mu1 z) Ta + b0 (1 - lambda2 Sa/2 - mu2 z) Sa - nu Ta Sa, b = -g rho'/rho0.
__device__ __forceinline__ double eos_buoyancy(const DevState& S, double T, double Sal, double z) {
    const double* e = S.eos;  // a0, b0, lambda1, lambda2, mu1, mu2, nu, t0, s0
    const double ta = T - e[7], sa = Sal - e[8];
    const double rho = -e[0] * (1.0 + 0.5 * e[2] * ta + e[4] * z) * ta + e[1] * (1.0 - 0.5 * e[3] * sa - e[5] * z) * sa -
                       e[6] * ta * sa;
    return -S.g * rho / S.rho0;
}

// N^2 on the face below layer k with salinity: both layers' buoyancy at the
// face's depth, differenced over the centre spacing.
__device__ __forceinline__ double eos_face_n2(const DevState& S, int k, double tk, double sk, double tb, double sb) {
    const double zf = S.zc[k] + 0.5 * S.dz[k];
    return (eos_buoyancy(S, tk, sk, zf) - eos_buoyancy(S, tb, sb, zf)) / S.dzc[k];
}

// Convective adjustment: from the state at the start of the step, kappa_conv
// on interior wet faces where the water above is denser than the water below
// (N^2 < 0: colder, with temperature alone), kappa0 on the other wet faces, 0
// on dry ones.
template <typename R>
__global__ __launch_bounds__(FW) void k_convective(const DevState S, double kappa_conv, double kappa0) {
    const int i = blockIdx.x * FW + threadIdx.x, j = blockIdx.y;
    if (i >= S.nx) return;
    const int nz = S.nz;
    const int kbot = nz - S.kb[idxk(S, i, j)];
    const R* T = f3<R>(S.t);
    const R* Sf = f3<R>(S.s);
    R* kw = f3<R>(S.kw);
    double below = 0.0, sbelow = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double tk = (k >= kbot) ? double(T[idx3(S, i, j, k)]) + S.tref[k] : 0.0;
        const double sk = (S.salinity && k >= kbot) ? double(Sf[idx3(S, i, j, k)]) + S.sref[k] : 0.0;
        bool unstable = false;
        if (k > kbot) unstable = S.salinity ? eos_face_n2(S, k, tk, sk, below, sbelow) < 0.0 : tk < below;
        const R val = (k > kbot) ? R(unstable ? kappa_conv : kappa0) : R(0);
        kw[idx3(S, i, j, k)] = val;
        for_each_image(S, i, j, S.h, [&](int x, int y) { kw[idx3(S, x, y, k)] = val; });
        below = tk;
        sbelow = sk;
    }
}

// Richardson-number mixing (Sec. 6 runs a Richardson-number-based mixing
// parameterization without giving its form; the Pacanowski-Philander form is
// the reading): on an interior wet face k, from the state at the start of
// the step, N^2 = g alpha dT/dz (with salinity, the buoyancy difference of the
// two layers at the face's depth over the centre spacing) and S^2 = |d(u_c, v_c)/dz|^2 with the
// velocities averaged to the cell centre; where N^2 < 0 both coefficients are
// conv, else with Ri = N^2 / max(S^2, 1e-16) and r = 1 / (1 + alpha Ri) the
// viscosity is nu0 r^2 + nu_b and the diffusivity nu r + kappa_b. Dry faces
// take 0. 256 adjacent columns per workgroup, one thread per column marching
// up the levels (loads issued eight levels at a time) with the lower level's
// values carried in registers.
constexpr int RW = 256;

template <typename R>
__global__ __launch_bounds__(RW) void k_richardson(const DevState S, const RiParams P) {
    const int i = blockIdx.x * RW + threadIdx.x, j = blockIdx.y;
    if (i >= S.nx) return;
    const int nz = S.nz;
    const int K = S.kb[idxk(S, i, j)];
    const int kbot = nz - K;
    const int ie = (i + 1 < S.nx) ? i + 1 : (S.periodic_x ? 0 : -1);
    const int jn = (j + 1 < S.ny) ? j + 1 : (S.periodic_y ? 0 : -1);
    const int Kuw = min(K, S.kb[idxk(S, i - 1, j)]);
    const int Kue = ie >= 0 ? min(K, S.kb[idxk(S, ie, j)]) : 0;
    const int Kvs = min(K, S.kb[idxk(S, i, j - 1)]);
    const int Kvn = jn >= 0 ? min(K, S.kb[idxk(S, i, jn)]) : 0;
    const int iec = ie >= 0 ? ie : i, jnc = jn >= 0 ? jn : j;
    const R* T = f3<R>(S.t);
    const R* Sf = f3<R>(S.s);
    const R* U = f3<R>(S.u);
    const R* V = f3<R>(S.v);
    R* kw = f3<R>(S.kw);
    R* kv = f3<R>(S.kv);
    const double ga = S.g * S.alpha;
    double tb = 0.0, sb = 0.0, ub = 0.0, vb = 0.0;  // the level below
    constexpr int CH = 8;                 // levels whose loads are issued together
    for (int k0 = 0; k0 < nz; k0 += CH) {
        R lT[CH], lUw[CH], lUe[CH], lVs[CH], lVn[CH], lS[CH];
#pragma unroll
        for (int m = 0; m < CH; ++m) {
            const int k = min(k0 + m, nz - 1);  // clamped: valid addresses, results unused past nz
            lT[m] = T[idx3(S, i, j, k)];
            lS[m] = S.salinity ? Sf[idx3(S, i, j, k)] : R(0);
            lUw[m] = U[idx3(S, i, j, k)];
            lUe[m] = U[idx3(S, iec, j, k)];
            lVs[m] = V[idx3(S, i, j, k)];
            lVn[m] = V[idx3(S, i, jnc, k)];
        }
#pragma unroll
        for (int m = 0; m < CH; ++m) {
            const int k = k0 + m;
            if (k >= nz) break;
            double kap = 0.0, nu = 0.0;
            if (k >= kbot) {
                const double tk = double(lT[m]) + S.tref[k];
                const double sk = S.salinity ? double(lS[m]) + S.sref[k] : 0.0;
                const double uw = (k >= nz - Kuw) ? double(lUw[m]) : 0.0;
                const double ue = (k >= nz - Kue) ? double(lUe[m]) : 0.0;
                const double vs = (k >= nz - Kvs) ? double(lVs[m]) : 0.0;
                const double vn = (k >= nz - Kvn) ? double(lVn[m]) : 0.0;
                const double uk = 0.5 * (uw + ue), vk = 0.5 * (vs + vn);
                if (k > kbot) {
                    const double dzc = S.dzc[k];
                    const double n2 = S.salinity ? eos_face_n2(S, k, tk, sk, tb, sb) : ga * (tk - tb) / dzc;
                    const double du = uk - ub, dv = vk - vb;
                    const double s2 = (du * du + dv * dv) / (dzc * dzc);
                    if (n2 < 0.0) {
                        kap = P.conv;
                        nu = P.conv;
                    } else {
                        const double ri = n2 / fmax(s2, 1e-16);
                        const double r = 1.0 / (1.0 + P.alpha * ri);
                        nu = P.nu0 * r * r + P.nu_b;
                        kap = nu * r + P.kappa_b;
                    }
                }
                tb = tk;
                sb = sk;
                ub = uk;
                vb = vk;
            }
            const R vkap = R(kap), vnu = R(nu);
            kw[idx3(S, i, j, k)] = vkap;
            kv[idx3(S, i, j, k)] = vnu;
            for_each_image(S, i, j, S.h, [&](int x, int y) {
                kw[idx3(S, x, y, k)] = vkap;
                kv[idx3(S, x, y, k)] = vnu;
            });
        }
    }
}

template <typename R>
hipError_t launch_richardson(const DevState& s, const RiParams& p, hipStream_t st) {
    if (!s.kw || !s.kv) return hipErrorInvalidValue;
    dim3 grid((s.nx + RW - 1) / RW, s.ny);
    hipLaunchKernelGGL(k_richardson<R>, grid, dim3(RW), 0, st, s, p);
    return hipGetLastError();
}
template hipError_t launch_richardson<double>(const DevState&, const RiParams&, hipStream_t);
template hipError_t launch_richardson<float>(const DevState&, const RiParams&, hipStream_t);

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
    const size_t lds = out_bf16 ? (size_t)FW * (din + 2) * 2 : features_lds(din);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    dim3 grid((s.nx + FW - 1) / FW, s.ny);
    if (out_bf16)
        hipLaunchKernelGGL((k_features<R, uint16_t>), grid, dim3(FW, FG), lds, st, s, din, norm,
                           static_cast<uint16_t*>(out));
    else
        hipLaunchKernelGGL((k_features<R, float>), grid, dim3(FW, FG), lds, st, s, din, norm, static_cast<float*>(out));
    return hipGetLastError();
}

template <typename R>
hipError_t launch_kappa_map(const DevState& s, const float* Y, int ldy, double kappa0, hipStream_t st) {
    const size_t lds = (size_t)FW * (s.nz + 1) * sizeof(float);
    dim3 grid((s.nx + FW - 1) / FW, s.ny);
    hipLaunchKernelGGL(k_kappa_map<R>, grid, dim3(FW, FG), lds, st, s, Y, ldy, kappa0);
    return hipGetLastError();
}

template hipError_t launch_features<double>(const DevState&, int, const float*, void*, int, hipStream_t);
template hipError_t launch_features<float>(const DevState&, int, const float*, void*, int, hipStream_t);
template hipError_t launch_kappa_map<double>(const DevState&, const float*, int, double, hipStream_t);
template hipError_t launch_kappa_map<float>(const DevState&, const float*, int, double, hipStream_t);

}  // namespace ocn
