// k_column.hip -- implicit vertical diffusion and the depth-mean correction.
//
// Backward-Euler vertical diffusion (paper Sec. 5.2: vertically implicit
// diffusion with a tridiagonal solver) of T, u and v, one thread per column,
// 256 adjacent columns per workgroup so that every level of a field is read
// and written as coalesced 1 KiB row segments.
//
// With a constant diffusivity the wet layers of T, u and v columns all start at
// the surface, so eliminating from the surface down gives pivots that do not
// depend on the column's depth except in its bottom layer: one level table
// built once on the host serves every column. The whole column is held in
// registers: the kernel is instantiated for a few level counts (NZB >= nz) and
// every loop over levels is unrolled, so the column's nz loads are all in
// flight at once and no LDS limits the number of resident waves. The
// temperature anomaly solve carries the diffusion of the reference profile on
// its right-hand side.
//
// For u and v the same kernel then applies the split-explicit correction
// (paper Sec. 5.3): the depth mean of u** is replaced by Ubar/H, the substep
// average of the barotropic transport (the transport that moved the free
// surface over the step), and it leaves the column
// sum sum_k dz u m_u of the stored result, which seeds the vertical transport
// of the next step. Columns next to a periodic boundary also write their
// wrapped copies into the halo.
#include "ocn_dev.h"

#include <algorithm>

namespace ocn {

constexpr int CW = 256;      // columns per workgroup of the single-state launches (four waves side by side
                             // read 1 KiB runs of each level: about 1.5x the rate of one-wave groups)
constexpr int CWB = 64;      // columns per tile of the batched ensemble launches (tile tables use 64)
constexpr int CWL = 64;      // columns per workgroup of the LDS-staged variable-diffusivity solve

template <typename R>
__device__ __forceinline__ void store_wrapped(const DevState& S, R* f, int i, int j, int k, R val) {
    for_each_image(S, i, j, S.h, [&](int x, int y) { f[idx3(S, x, y, k)] = val; });
}

__device__ __forceinline__ void store_wrapped2(const DevState& S, double* f, int i, int j, double val) {
    f[idx2(S, i, j)] = val;
    for_each_image(S, i, j, S.h, [&](int x, int y) { f[idx2(S, x, y)] = val; });
}

// Level-count buckets of the register-resident solve.
constexpr int kNzBuckets[] = {16, 32, 48, 64, 80, 100, 128};
constexpr int kMaxNz = kMaxLevels;

// Copy a stored column into its periodic images (edge columns only): the
// values are read back from the column just written by this thread, so the
// unrolled level loops above keep the column in registers.
template <typename R>
__device__ __forceinline__ void copy_images(const DevState& S, R* dst, int i, int j) {
    const Images im = column_images(S, i, j, S.h);
    if (im.n == 0) return;
    const long long o0 = idx3(S, i, j, 0), pl = S.plane3;
    for (int k = 0; k < S.nz; ++k) {
        const long long o = o0 + k * pl;
        const R val = dst[o];
        if (im.n > 3) {
            store_wrapped(S, dst, i, j, k, val);
            continue;
        }
        dst[o + im.o0] = val;
        if (im.n > 1) {
            dst[o + im.o1] = val;
            dst[o + im.o2] = val;
        }
    }
}

// Field of a column solve and its predicted source: 0 = T, 1 = u, 2 = v, 3 = S.
template <typename R>
__device__ __forceinline__ R* col_dst(const DevState& S, int field) {
    return f3<R>(field == 0 ? S.t : field == 1 ? S.u : field == 2 ? S.v : S.s);
}
template <typename R>
__device__ __forceinline__ const R* col_src(const DevState& S, int field) {
    return f3<R>(field == 0 ? S.ts : field == 1 ? S.us : field == 2 ? S.vs : S.ss);
}

// Output of one solved column: T and S as they are; u and v with the depth-mean
// correction u = u** + (Ubar - sum dz u**) / H on wet layers, which also
// leaves the column sum sum_k dz u m_u of the stored result (it seeds the
// vertical transport of the next step). Periodic images are written too.
template <typename R, int NZB>
__device__ __forceinline__ void column_store(const DevState& S, const R (&x)[NZB], const int i, const int j,
                                             const int field, const int kbot, const double colsum) {
    const int nz = S.nz;
    R* dst = col_dst<R>(S, field);
    const long long o0 = idx3(S, i, j, 0), pl = S.plane3;
    if (field == 0 || field == 3) {
        R* q = dst + o0;
#pragma unroll
        for (int k = 0; k < NZB; ++k) {
            if (k < nz) *q = x[k];
            q += pl;
        }
        copy_images(S, dst, i, j);
        return;
    }
    const double H = (field == 1) ? S.hu[idx2(S, i, j)] : S.hv[idx2(S, i, j)];
    const double B = (field == 1) ? S.ubt_mean[idx2(S, i, j)] : S.vbt_mean[idx2(S, i, j)];  // substep-averaged transport
    const double corr = (H > 0.0) ? (B - colsum) / H : 0.0;
    double newsum = 0.0;
    R* q = dst + o0;
#pragma unroll
    for (int k = 0; k < NZB; ++k) {
        if (k < nz) {
            R val = R(0);
            if (k >= kbot && H > 0.0) {
                val = R(double(x[k]) + corr);
                newsum += double(S.dz[k]) * double(val);
            }
            *q = val;
        }
        q += pl;
    }
    copy_images(S, dst, i, j);
    store_wrapped2(S, field == 1 ? S.cu : S.cv, i, j, newsum);
}

// One block of W columns (bx, j) of one field: 0 = T, 1 = u, 2 = v, 3 = S.
// Backward Euler with the constant diffusivity, eliminated from the surface
// down: r'_k = r_k - (c_k / b'_{k+1}) r'_{k+1}, then from the bottom layer up
// x_k = (r'_k - a_k x_{k-1}) / b'_k, the bottom layer with its own pivot b''.
// Every coefficient is uniform across the wave (a level table), so the
// column's only memory traffic is its own values.
template <typename R, int NZB, int W>
__device__ __forceinline__ void column_regs(const DevState& S, const int bx, const int j, const int field) {
    const int t = threadIdx.x;
    const int i = bx * W + t;
    const int nz = S.nz;
    const int ic = i < S.nx ? i : S.nx - 1;

    const int kc = S.kb[idxk(S, ic, j)];
    int K = kc;
    if (field == 1) K = min(kc, S.kb[idxk(S, ic - 1, j)]);
    if (field == 2) K = min(kc, S.kb[idxk(S, ic, j - 1)]);
    const int kbot = nz - K;  // lowest wet layer
    const bool mom = field == 1 || field == 2;

    const R* src = col_src<R>(S, field) + idx3(S, ic, j, 0);
    const R* tab = static_cast<const R*>(S.thomas_tab);
    const R* dtr = static_cast<const R*>(field == 3 ? S.dsr : S.dtr);
    const long long pl = S.plane3;

    R x[NZB];
    {
        const R* q = src;
#pragma unroll
        for (int k = 0; k < NZB; ++k) {
            x[k] = (k < nz) ? *q : R(0);
            q += pl;
        }
    }

    // Right-hand sides of the wet layers (dry layers keep phi*). Temperature
    // is stored as T' = T - tref(k): diffusing T is diffusing T' with
    // dt dz L(tref) = -c_k (tref_{k+1} - tref_k) + a_k (tref_k - tref_{k-1})
    // added to its right-hand side.
#pragma unroll
    for (int k = 0; k < NZB; ++k) {
        if (k < nz && k >= kbot) {
            R rhs = R(S.dz[k]) * x[k];
            if (!mom) {
                const R a = (k > kbot) ? tab[4 * k + 3] : R(0);         // face k wet: layers k-1 and k
                const R c = (k < nz - 1) ? tab[4 * (k + 1) + 3] : R(0);  // face k+1
                rhs += -c * dtr[k * 4 + 2] - a * dtr[k * 4 + 1];
            }
            x[k] = rhs;
        }
    }
    // elimination from the surface down
    R rn = R(0);
#pragma unroll
    for (int k = NZB - 1; k >= 0; --k) {
        if (k < nz && k >= kbot) {
            rn = fma(-tab[4 * k + 1], rn, x[k]);
            x[k] = rn;
        }
    }
    // substitution from the bottom layer up
    R xp = R(0);
    double colsum = 0.0;
#pragma unroll
    for (int k = 0; k < NZB; ++k) {
        if (k < nz && k >= kbot) {
            xp = (k == kbot) ? x[k] * tab[4 * k + 2] : (x[k] - tab[4 * k + 3] * xp) * tab[4 * k];
            x[k] = xp;
            colsum += double(S.dz[k]) * double(xp);
        }
    }
    if (i < S.nx) column_store<R, NZB>(S, x, i, j, field, kbot, colsum);
}

// The same solve with a diffusivity that varies by face and column (a
// prescribed field or the learned closure): the tridiagonal coefficients are
// formed on the fly, a_k = -dt kappa_k / dzc_k on the wet face k below layer
// k, c_k = a_{k+1}; the eliminated super-diagonal c' is kept in a second LDS
// array. u and v take the mean of the two neighbouring tracer-face values.
template <typename R, int W>
__device__ __forceinline__ void column_block_vk(const DevState& S, R* sd, R* sc, const int bx, const int j,
                                                const int field) {
    const int t = threadIdx.x;
    const int i = bx * W + t;
    const int nz = S.nz;
    const bool live = i < S.nx;
    const int ic = live ? i : S.nx - 1;

    const int kc = S.kb[idxk(S, ic, j)];
    int K = kc;
    if (field == 1) K = min(kc, S.kb[idxk(S, ic - 1, j)]);
    if (field == 2) K = min(kc, S.kb[idxk(S, ic, j - 1)]);
    const bool mom = field == 1 || field == 2;

    const R* src = col_src<R>(S, field) + idx3(S, ic, j, 0);
    R* dst = col_dst<R>(S, field);
    const R* dtr = static_cast<const R*>(field == 3 ? S.dsr : S.dtr);
    const R* kwf = static_cast<const R*>(mom && S.kv ? S.kv : S.kw);  // u, v: viscosity when set
    const long long o0 = idx3(S, ic, j, 0);
    const long long on = field == 1 ? idx3(S, ic - 1, j, 0) : idx3(S, ic, j - 1, 0);
    const int kbot = nz - K;
    const long long pl = S.plane3;
    const R rdt = R(S.dt);

    auto coef = [&](int k) -> R {  // a_k of face k, 0 unless the face is wet
        if (k <= kbot || k >= nz) return R(0);
        R kap = kwf[o0 + k * pl];
        if (mom) kap = R(0.5) * (kwf[on + k * pl] + kap);
        return -rdt * kap / R(S.dzc[k]);
    };

    // stage the column and its face coefficients (sc holds a_k until the
    // elimination overwrites it with c'_k)
#pragma unroll 8
    for (int k = 0; k < nz; ++k) {
        sd[k * W + t] = src[k * pl];
        sc[k * W + t] = coef(k);
    }

    R dprev = R(0), cprev = R(0), ak = R(0);
    for (int k = 0; k < nz; ++k) {
        const R ck = (k + 1 < nz) ? sc[(k + 1) * W + t] : R(0);
        R rhs = R(S.dz[k]) * sd[k * W + t];
        if (!mom) rhs += -ck * dtr[k * 4 + 2] - ak * dtr[k * 4 + 1];
        const R rden = R(1) / (R(S.dz[k]) - ak - ck - ak * cprev);
        const R cpk = ck * rden;
        const R dk = (rhs - ak * dprev) * rden;
        sd[k * W + t] = dk;
        sc[k * W + t] = cpk;
        dprev = dk;
        cprev = cpk;
        ak = ck;
    }
    R xnext = R(0);
    double colsum = 0.0;
    for (int k = nz - 1; k >= 0; --k) {
        const R x = sd[k * W + t] - sc[k * W + t] * xnext;
        xnext = x;
        sd[k * W + t] = x;
        if (k >= kbot) colsum += double(S.dz[k]) * double(x);
    }
    if (!live) return;

    if (!mom) {
        for (int k = 0; k < nz; ++k) {
            const R x = sd[k * W + t];
            dst[idx3(S, i, j, k)] = x;
            store_wrapped(S, dst, i, j, k, x);
        }
        return;
    }
    const double H = (field == 1) ? S.hu[idx2(S, i, j)] : S.hv[idx2(S, i, j)];
    const double B = (field == 1) ? S.ubt_mean[idx2(S, i, j)] : S.vbt_mean[idx2(S, i, j)];  // substep-averaged transport
    const double corr = (H > 0.0) ? (B - colsum) / H : 0.0;
    double newsum = 0.0;
    for (int k = 0; k < nz; ++k) {
        R val = R(0);
        if (k >= kbot && H > 0.0) {
            val = R(double(sd[k * W + t]) + corr);
            newsum += double(S.dz[k]) * double(val);
        }
        dst[idx3(S, i, j, k)] = val;
        store_wrapped(S, dst, i, j, k, val);
    }
    store_wrapped2(S, field == 1 ? S.cu : S.cv, i, j, newsum);
}

// Reciprocal on the serial elimination chain: the hardware estimate in FP32
// (1 ulp), the correctly rounded division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Register-resident form of the variable-diffusivity solve, for columns whose
// values and coefficients fit the registers (FP32 up to 100 levels, FP64 up to
// 32): the column and its face coefficients a_k are loaded up front (all loads
// in flight together), and c'_k overwrites a_k once level k is eliminated.
// The arithmetic is that of column_block_vk, level by level.
template <typename R, int NZB, int W>
__device__ __forceinline__ void column_regs_vk(const DevState& S, const int bx, const int j, const int field) {
    const int t = threadIdx.x;
    const int i = bx * W + t;
    const int nz = S.nz;
    const int ic = i < S.nx ? i : S.nx - 1;

    const int kc = S.kb[idxk(S, ic, j)];
    int K = kc;
    if (field == 1) K = min(kc, S.kb[idxk(S, ic - 1, j)]);
    if (field == 2) K = min(kc, S.kb[idxk(S, ic, j - 1)]);
    const int kbot = nz - K;
    const bool mom = field == 1 || field == 2;

    const R* src = col_src<R>(S, field) + idx3(S, ic, j, 0);
    const R* kwf = static_cast<const R*>(mom && S.kv ? S.kv : S.kw);  // u, v: viscosity when set
    const R* dtr = static_cast<const R*>(field == 3 ? S.dsr : S.dtr);
    const long long o0 = idx3(S, ic, j, 0);
    const long long on = field == 1 ? idx3(S, ic - 1, j, 0) : idx3(S, ic, j - 1, 0);
    const long long pl = S.plane3;
    const R rdt = R(S.dt);

    R x[NZB], a[NZB];
    {
        const R* qx = src;
        const R* qk = kwf + o0;
        const R* qn = kwf + on;
#pragma unroll
        for (int k = 0; k < NZB; ++k) {
            x[k] = (k < nz) ? *qx : R(0);
            a[k] = R(0);
            if (k < nz && k > kbot) {  // face k wet: layers k-1 and k
                R kap = *qk;
                if (mom) kap = R(0.5) * (*qn + kap);
                a[k] = -rdt * kap / R(S.dzc[k]);
            }
            qx += pl;
            qk += pl;
            qn += pl;
        }
    }
    R dprev = R(0), cprev = R(0);
#pragma unroll
    for (int k = 0; k < NZB; ++k) {
        if (k < nz) {
            const R ak = a[k];
            const R ck = (k + 1 < NZB) ? a[k + 1 < NZB ? k + 1 : k] : R(0);  // a_{k+1} (0 above the top)
            R rhs = R(S.dz[k]) * x[k];
            if (!mom) rhs += -ck * dtr[k * 4 + 2] - ak * dtr[k * 4 + 1];
            const R rden = recip(R(S.dz[k]) - ak - ck - ak * cprev);
            cprev = ck * rden;
            dprev = (rhs - ak * dprev) * rden;
            x[k] = dprev;
            a[k] = cprev;
        }
    }
    R xnext = R(0);
    double colsum = 0.0;
#pragma unroll
    for (int k = NZB - 1; k >= 0; --k) {
        if (k < nz) {
            xnext = x[k] - a[k] * xnext;
            x[k] = xnext;
            if (k >= kbot) colsum += double(S.dz[k]) * double(xnext);
        }
    }
    if (i < S.nx) column_store<R, NZB>(S, x, i, j, field, kbot, colsum);
}

// Column sums sum_k dz u m_u and sum_k dz v m_v of the stored velocities (used
// after u or v is set from the host).
template <typename R>
__global__ __launch_bounds__(CW) void k_colsum(const DevState S) {
    const int i = blockIdx.x * CW + threadIdx.x, j = blockIdx.y, field = blockIdx.z;
    if (i >= S.nx) return;
    const int kc = S.kb[idxk(S, i, j)];
    const int K = (field == 0) ? min(kc, S.kb[idxk(S, i - 1, j)]) : min(kc, S.kb[idxk(S, i, j - 1)]);
    const R* f = f3<R>(field == 0 ? S.u : S.v);
    double s = 0.0;
    for (int k = S.nz - K; k < S.nz; ++k) s += double(S.dz[k]) * double(f[idx3(S, i, j, k)]);
    store_wrapped2(S, field == 0 ? S.cu : S.cv, i, j, s);
}

// Vertical velocity on every z-face from continuity, integrated upward from the
// bottom (a diagnostic output; faces 0..nz-1 into ts, the surface face into scratch2d).
template <typename R>
__global__ __launch_bounds__(CW) void k_wfaces(const DevState S) {
    const int i = blockIdx.x * CW + threadIdx.x, j = blockIdx.y;
    if (i >= S.nx) return;
    const int nz = S.nz;
    const int* kb = S.kb;
    const int K0 = kb[idxk(S, i, j)];
    const int Ku0 = min(kb[idxk(S, i - 1, j)], K0), Ku1 = min(K0, kb[idxk(S, i + 1, j)]);
    const int Kv0 = min(kb[idxk(S, i, j - 1)], K0), Kv1 = min(K0, kb[idxk(S, i, j + 1)]);
    const R* u = f3<R>(S.u);
    const R* v = f3<R>(S.v);
    R* out = f3<R>(S.ts);
    const double area = S.area[j];
    double W = 0.0;
    for (int k = 0; k < nz; ++k) {
        out[idx3(S, i, j, k)] = R(W / area);
        const int kw = nz - k;
        const double dz = S.dz[k];
        const double ue = (Ku1 >= kw) ? double(u[idx3(S, i + 1, j, k)]) * S.dy * dz : 0.0;
        const double uw = (Ku0 >= kw) ? double(u[idx3(S, i, j, k)]) * S.dy * dz : 0.0;
        const double vn = (Kv1 >= kw) ? double(v[idx3(S, i, j + 1, k)]) * S.dxv[j + 1] * dz : 0.0;
        const double vs = (Kv0 >= kw) ? double(v[idx3(S, i, j, k)]) * S.dxv[j] * dz : 0.0;
        W = W - (ue - uw + vn - vs);
    }
    S.scratch2d[idx2(S, i, j)] = W / area;
}

// Occupancy target of the register-resident solve: FP32 columns of up to 100
// levels fit four waves per SIMD.
template <typename R> struct ColWaves;
template <> struct ColWaves<float> { static constexpr int n = 4; };
template <> struct ColWaves<double> { static constexpr int n = 2; };

template <typename R, int NZB>
__global__ __launch_bounds__(CW) __attribute__((amdgpu_waves_per_eu(ColWaves<R>::n)))
void k_column(const DevState S) {
    column_regs<R, NZB, CW>(S, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Register-resident variable-diffusivity solve: two column arrays per thread.
template <typename R, int NZB> struct VkWaves { static constexpr int n = (sizeof(R) == 4 && NZB <= 48) ? 4 : 2; };
template <typename R, int NZB> struct VkRegs { static constexpr bool ok = sizeof(R) == 4 ? NZB <= 100 : NZB <= 32; };

template <typename R, int NZB>
__global__ __launch_bounds__(CW) __attribute__((amdgpu_waves_per_eu(VkWaves<R, NZB>::n)))
void k_column_vkr(const DevState S) {
    column_regs_vk<R, NZB, CW>(S, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Variable diffusivity (prescribed field or learned closure), staged in LDS,
// W columns per workgroup (32 when 64 columns of the two arrays exceed 64 KB).
template <typename R, int W>
__global__ __launch_bounds__(W) void k_column_vk(const DevState S) {
    extern __shared__ __align__(16) unsigned char smem_col[];
    R* sd = reinterpret_cast<R*>(smem_col);  // nz * W eliminated rhs / solution, then nz * W of c'
    column_block_vk<R, W>(S, sd, sd + S.nz * W, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Ensemble: entry blockIdx.x of the table is (member, bx, j); blockIdx.y is the field.
template <typename R, int NZB>
__global__ __launch_bounds__(CWB) __attribute__((amdgpu_waves_per_eu(ColWaves<R>::n)))
void k_column_batched(const DevState* __restrict__ members, const int4* __restrict__ tiles) {
    const int4 e = tiles[blockIdx.x];
    column_regs<R, NZB, CWB>(members[e.x], e.y, e.z, blockIdx.y);
}

// The same over a queue of (table entry, field) items, field-major, with
// persistent workgroups.
template <typename R, int NZB>
__global__ __launch_bounds__(CWB) __attribute__((amdgpu_waves_per_eu(ColWaves<R>::n)))
void k_column_queued(const DevState* __restrict__ members, const int4* __restrict__ tiles, const int ntiles,
                     int* __restrict__ queue) {
    for_each_queued_tile(queue, 3 * ntiles, [&](int i) {
        const int field = i / ntiles;
        const int4 e = tiles[i - field * ntiles];
        column_regs<R, NZB, CWB>(members[e.x], e.y, e.z, field);
    });
}

// Dispatch a level count to the smallest bucket that holds it.
template <typename R, template <typename, int> class Launch, typename... A>
hipError_t with_bucket(int nz, A... args) {
    if (nz <= 16) return Launch<R, 16>::go(args...);
    if (nz <= 32) return Launch<R, 32>::go(args...);
    if (nz <= 48) return Launch<R, 48>::go(args...);
    if (nz <= 64) return Launch<R, 64>::go(args...);
    if (nz <= 80) return Launch<R, 80>::go(args...);
    if (nz <= 100) return Launch<R, 100>::go(args...);
    if (nz <= kMaxNz) return Launch<R, 128>::go(args...);
    return hipErrorInvalidValue;
}

template <typename R, int NZB>
struct LaunchColumn {
    static hipError_t go(const DevState& s, hipStream_t st) {
        dim3 grid((s.nx + CW - 1) / CW, s.ny, s.salinity ? 4 : 3);
        hipLaunchKernelGGL((k_column<R, NZB>), grid, dim3(CW), 0, st, s);
        return hipGetLastError();
    }
};

template <typename R, int NZB>
struct LaunchColumnVk {
    static hipError_t go(const DevState& s, hipStream_t st) {
        dim3 grid((s.nx + CW - 1) / CW, s.ny, s.salinity ? 4 : 3);
        if constexpr (VkRegs<R, NZB>::ok) {
            hipLaunchKernelGGL((k_column_vkr<R, NZB>), grid, dim3(CW), 0, st, s);
        } else {
            const size_t lds = (size_t)s.nz * CWL * sizeof(R) * 2;
            if (lds <= 64 * 1024) {
                dim3 g1((s.nx + CWL - 1) / CWL, s.ny, s.salinity ? 4 : 3);
                hipLaunchKernelGGL((k_column_vk<R, CWL>), g1, dim3(CWL), lds, st, s);
            } else {
                if (lds / 2 > 64 * 1024) return hipErrorInvalidValue;  // per-workgroup LDS limit
                dim3 g2((s.nx + CWL / 2 - 1) / (CWL / 2), s.ny, s.salinity ? 4 : 3);
                hipLaunchKernelGGL((k_column_vk<R, CWL / 2>), g2, dim3(CWL / 2), lds / 2, st, s);
            }
        }
        return hipGetLastError();
    }
};

template <typename R, int NZB>
struct LaunchColumnBatched {
    static hipError_t go(const DevState* members, const int4* tiles, int ntiles, int* queue, hipStream_t st) {
        if (queue) {
            const int nb = std::min(3 * ntiles, resident_workgroups((const void*)k_column_queued<R, NZB>, CWB));
            hipLaunchKernelGGL((k_column_queued<R, NZB>), dim3(nb), dim3(CWB), 0, st, members, tiles, ntiles, queue);
        } else {
            hipLaunchKernelGGL((k_column_batched<R, NZB>), dim3(ntiles, 3), dim3(CWB), 0, st, members, tiles);
        }
        return hipGetLastError();
    }
};

template <typename R>
hipError_t launch_column_batched(const DevState* members, const int4* tiles, int ntiles, int max_nz, int* queue,
                                 hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    return with_bucket<R, LaunchColumnBatched>(max_nz, members, tiles, ntiles, queue, st);
}

template hipError_t launch_column_batched<double>(const DevState*, const int4*, int, int, int*, hipStream_t);
template hipError_t launch_column_batched<float>(const DevState*, const int4*, int, int, int*, hipStream_t);

template <typename R>
hipError_t launch_column(const DevState& s, hipStream_t st) {
    if (s.kw) return with_bucket<R, LaunchColumnVk>(s.nz, s, st);
    return with_bucket<R, LaunchColumn>(s.nz, s, st);
}

template <typename R>
hipError_t launch_colsum(const DevState& s, hipStream_t st) {
    dim3 grid((s.nx + CW - 1) / CW, s.ny, 2);
    hipLaunchKernelGGL(k_colsum<R>, grid, dim3(CW), 0, st, s);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_w_faces(const DevState& s, double* /*unused*/, hipStream_t st) {
    dim3 grid((s.nx + CW - 1) / CW, s.ny, 1);
    hipLaunchKernelGGL(k_wfaces<R>, grid, dim3(CW), 0, st, s);
    return hipGetLastError();
}

template hipError_t launch_column<double>(const DevState&, hipStream_t);
template hipError_t launch_column<float>(const DevState&, hipStream_t);
template hipError_t launch_colsum<double>(const DevState&, hipStream_t);
template hipError_t launch_colsum<float>(const DevState&, hipStream_t);
template hipError_t launch_w_faces<double>(const DevState&, double*, hipStream_t);
template hipError_t launch_w_faces<float>(const DevState&, double*, hipStream_t);

}  // namespace ocn
