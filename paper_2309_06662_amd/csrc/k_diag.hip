// k_diag.hip -- diagnostics reductions.
//
// Tracer content, free-surface volume, kinetic energy, extrema, the advective
// CFL number and a count of non-finite values, reduced on the device.
// Sums are compensated (Neumaier) in FP64 for every precision: per thread
// over its column, across the 64 lanes of a wavefront by butterfly shuffles,
// across the wavefronts of a workgroup through LDS, then one partial per
// workgroup into fixed slots that a single-workgroup pass reduces in index
// order, so the result does not depend on scheduling.
#include "ocn_dev.h"

#include <mutex>

namespace ocn {

constexpr int DX = 64, DY = 4, DT = DX * DY;

struct Acc {
    double s[DG_NSUM], c[DG_NSUM];
    double m[DG_NONFINITE - DG_NSUM];
    double nonfinite;
};

__device__ __forceinline__ void two_sum_add(double& s, double& c, double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
}

__device__ __forceinline__ void combine(Acc& a, const Acc& b) {
    for (int q = 0; q < DG_NSUM; ++q) {
        two_sum_add(a.s[q], a.c[q], b.s[q]);
        a.c[q] += b.c[q];
    }
    for (int q = 0; q < DG_NONFINITE - DG_NSUM; ++q) a.m[q] = fmax(a.m[q], b.m[q]);
    a.nonfinite += b.nonfinite;
}

__device__ __forceinline__ void shfl_acc(Acc& o, const Acc& a, int lanemask) {
    for (int q = 0; q < DG_NSUM; ++q) {
        o.s[q] = __shfl_xor(a.s[q], lanemask);
        o.c[q] = __shfl_xor(a.c[q], lanemask);
    }
    for (int q = 0; q < DG_NONFINITE - DG_NSUM; ++q) o.m[q] = __shfl_xor(a.m[q], lanemask);
    o.nonfinite = __shfl_xor(a.nonfinite, lanemask);
}

__device__ void block_reduce_store(Acc& a, double* out) {
    // wavefront butterfly
    for (int mask = 32; mask >= 1; mask >>= 1) {
        Acc o;
        shfl_acc(o, a, mask);
        combine(a, o);
    }
    __shared__ double sh[DT / 64][DG_COUNT + DG_NSUM];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    if (lane == 0) {
        for (int q = 0; q < DG_NSUM; ++q) { sh[wave][q] = a.s[q]; sh[wave][DG_COUNT + q] = a.c[q]; }
        for (int q = DG_NSUM; q < DG_NONFINITE; ++q) sh[wave][q] = a.m[q - DG_NSUM];
        sh[wave][DG_NONFINITE] = a.nonfinite;
    }
    __syncthreads();
    if (tid == 0) {
        Acc r;
        for (int q = 0; q < DG_NSUM; ++q) { r.s[q] = sh[0][q]; r.c[q] = sh[0][DG_COUNT + q]; }
        for (int q = DG_NSUM; q < DG_NONFINITE; ++q) r.m[q - DG_NSUM] = sh[0][q];
        r.nonfinite = sh[0][DG_NONFINITE];
        for (int w = 1; w < DT / 64; ++w) {
            Acc b;
            for (int q = 0; q < DG_NSUM; ++q) { b.s[q] = sh[w][q]; b.c[q] = sh[w][DG_COUNT + q]; }
            for (int q = DG_NSUM; q < DG_NONFINITE; ++q) b.m[q - DG_NSUM] = sh[w][q];
            b.nonfinite = sh[w][DG_NONFINITE];
            combine(r, b);
        }
        for (int q = 0; q < DG_NSUM; ++q) out[q] = r.s[q] + r.c[q];
        for (int q = DG_NSUM; q < DG_NONFINITE; ++q) out[q] = r.m[q - DG_NSUM];
        out[DG_NONFINITE] = r.nonfinite;
    }
}

__device__ __forceinline__ void init_acc(Acc& a) {
    for (int q = 0; q < DG_NSUM; ++q) { a.s[q] = 0.0; a.c[q] = 0.0; }
    for (int q = 0; q < DG_NONFINITE - DG_NSUM; ++q) a.m[q] = -INFINITY;
    a.nonfinite = 0.0;
}

template <typename R>
__global__ __launch_bounds__(DT) void k_diag_partial(const DevState S) {
    const int i = blockIdx.x * DX + threadIdx.x, j = blockIdx.y * DY + threadIdx.y;
    Acc a;
    init_acc(a);
    if (i < S.nx && j < S.ny) {
        const int nz = S.nz;
        const int K = S.kb[idxk(S, i, j)];
        const int Ku = min(K, S.kb[idxk(S, i - 1, j)]), Ku1 = min(K, S.kb[idxk(S, i + 1, j)]);
        const int Kv = min(K, S.kb[idxk(S, i, j - 1)]), Kv1 = min(K, S.kb[idxk(S, i, j + 1)]);
        const R* u = f3<R>(S.u);
        const R* v = f3<R>(S.v);
        const R* t = f3<R>(S.t);
        const R* sal = f3<R>(S.s);  // salinity only
        const double area = S.area[j], dxc = S.dxc[j], dxv = S.dxv[j], dy = S.dy, dt = S.dt;
        double W = 0.0;
        for (int k = 0; k < nz; ++k) {
            const long long o = idx3(S, i, j, k);
            const double uu = double(u[o]), vv = double(v[o]), tt = double(t[o]) + S.tref[k];
            const double ss = S.salinity ? double(sal[o]) + S.sref[k] : 0.0;
            if (!isfinite(uu) || !isfinite(vv) || !isfinite(tt) || !isfinite(ss)) a.nonfinite += 1.0;
            const int kw = nz - k;
            const double dz = S.dz[k];
            if (K >= kw) {
                two_sum_add(a.s[DG_TRACER], a.c[DG_TRACER], area * dz * tt);
                if (S.salinity) two_sum_add(a.s[DG_SALT], a.c[DG_SALT], area * dz * ss);
                a.m[DG_T_MAX - DG_NSUM] = fmax(a.m[DG_T_MAX - DG_NSUM], tt);
                a.m[DG_NEG_T_MIN - DG_NSUM] = fmax(a.m[DG_NEG_T_MIN - DG_NSUM], -tt);
            }
            double ke = 0.0;
            if (Ku >= kw) {
                ke += area * dz * uu * uu;
                a.m[DG_MAX_U - DG_NSUM] = fmax(a.m[DG_MAX_U - DG_NSUM], fabs(uu));
                a.m[DG_CFL - DG_NSUM] = fmax(a.m[DG_CFL - DG_NSUM], fabs(uu) * dt / dxc);
            }
            if (Kv >= kw) {
                ke += dxv * dy * dz * vv * vv;
                a.m[DG_MAX_V - DG_NSUM] = fmax(a.m[DG_MAX_V - DG_NSUM], fabs(vv));
                a.m[DG_CFL - DG_NSUM] = fmax(a.m[DG_CFL - DG_NSUM], fabs(vv) * dt / dy);
            }
            two_sum_add(a.s[DG_KE], a.c[DG_KE], 0.5 * ke);
            // vertical velocity on the bottom face of layer k, from the bottom up
            if (k >= 1 && K >= kw + 1) {
                const double wv = fabs(W / area);
                a.m[DG_MAX_W - DG_NSUM] = fmax(a.m[DG_MAX_W - DG_NSUM], wv);
                a.m[DG_CFL - DG_NSUM] = fmax(a.m[DG_CFL - DG_NSUM], wv * dt / S.dzc[k]);
            }
            const double ue = (Ku1 >= kw) ? double(u[idx3(S, i + 1, j, k)]) * dy * dz : 0.0;
            const double uw = (Ku >= kw) ? uu * dy * dz : 0.0;
            const double vn = (Kv1 >= kw) ? double(v[idx3(S, i, j + 1, k)]) * S.dxv[j + 1] * dz : 0.0;
            const double vs = (Kv >= kw) ? vv * dxv * dz : 0.0;
            W = W - (ue - uw + vn - vs);
        }
        const long long c2 = idx2(S, i, j);
        const double e = S.eta[c2];
        if (!isfinite(e) || !isfinite(S.ubt[c2]) || !isfinite(S.vbt[c2])) a.nonfinite += 1.0;
        if (K > 0) {
            two_sum_add(a.s[DG_VOLUME], a.c[DG_VOLUME], area * e);
            two_sum_add(a.s[DG_VOLUME_MEAN], a.c[DG_VOLUME_MEAN], area * S.eta_mean[c2]);
            two_sum_add(a.s[DG_WET_AREA], a.c[DG_WET_AREA], area);
            a.m[DG_ETA_MAX - DG_NSUM] = fmax(a.m[DG_ETA_MAX - DG_NSUM], e);
            a.m[DG_NEG_ETA_MIN - DG_NSUM] = fmax(a.m[DG_NEG_ETA_MIN - DG_NSUM], -e);
        }
    }
    const long long b = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    block_reduce_store(a, S.diag_part + b * DG_COUNT);
}

__global__ __launch_bounds__(DT) void k_diag_final(const DevState S, int nblocks) {
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    Acc a;
    init_acc(a);
    for (int b = tid; b < nblocks; b += DT) {
        const double* p = S.diag_part + (long long)b * DG_COUNT;
        Acc x;
        for (int q = 0; q < DG_NSUM; ++q) { x.s[q] = p[q]; x.c[q] = 0.0; }
        for (int q = DG_NSUM; q < DG_NONFINITE; ++q) x.m[q - DG_NSUM] = p[q];
        x.nonfinite = p[DG_NONFINITE];
        combine(a, x);
    }
    block_reduce_store(a, S.diag_out);
}

template <typename R>
hipError_t launch_diagnostics(const DevState& s, hipStream_t st) {
    dim3 block(DX, DY);
    dim3 grid((s.nx + DX - 1) / DX, (s.ny + DY - 1) / DY);
    const int nb = grid.x * grid.y;
    if (nb > s.diag_blocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_diag_partial<R>, grid, block, 0, st, s);
    hipLaunchKernelGGL(k_diag_final, dim3(1), block, 0, st, s, nb);
    return hipGetLastError();
}

template hipError_t launch_diagnostics<double>(const DevState&, hipStream_t);
template hipError_t launch_diagnostics<float>(const DevState&, hipStream_t);

// Fixed scratch of the no-allocation diagnostics: the per-workgroup partials
// of up to kDiagScratchBlocks workgroups (64 x 4 columns each, so grids of up
// to 8.4 million columns), then the DG_COUNT final values. Each GPU holds its
// own copy until the process ends; concurrent calls on one GPU share it.
constexpr int kDiagScratchBlocks = 32768;
static __device__ __align__(256) double scratch[(kDiagScratchBlocks + 1) * DG_COUNT];

// Device address of this GPU's scratch array, looked up once per device with
// that device current (host code never passes the symbol itself).
hipError_t diag_scratch(int device, double** ptr, int* max_blocks) {
    constexpr int kMaxDevices = 64;
    static double* addr[kMaxDevices] = {};
    static std::mutex lock;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double*>(p);
    }
    *ptr = addr[device];
    *max_blocks = kDiagScratchBlocks;
    return hipSuccess;
}

}  // namespace ocn
