// k_baro.hip -- the sub-cycled barotropic free-surface loop (paper Sec. 5.3).
//
// Forward-backward substeps in FP64 for every precision: the free surface
// first, from the divergence of the depth-integrated transports, then the
// transports from the new surface gradient plus the slow forcing left by the
// tendency kernel. Running sums of eta^{m+1}, U^m and V^m give the step
// averages. Each substep is two launches over the 2D grid (surface, then
// transports); every thread updates one column in place and writes the
// periodic copies of its value into the one-cell halo the next launch reads.
#include "ocn_dev.h"

namespace ocn {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ void wrap2(const DevState& S, double* f, int i, int j, double val) {
    // periodic copies into the halo band
    for_each_image(S, i, j, S.h, [&](int x, int y) { f[idx2(S, x, y)] = val; });
}

__global__ __launch_bounds__(BX * BY) void k_baro_eta(const DevState S, const double dtau, const int m) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= S.nx || j >= S.ny) return;
    const long long c = idx2(S, i, j);
    const double Uc = S.ubt[c], Vc = S.vbt[c];
    const double div = S.dy * (S.ubt[c + 1] - Uc) + S.dxv[j + 1] * S.vbt[c + S.p2] - S.dxv[j] * Vc;
    const double e = S.eta[c] - dtau / S.area[j] * div;
    S.eta[c] = e;
    wrap2(S, S.eta, i, j, e);
    if (m == 0) {
        S.se[c] = e;
        S.su[c] = Uc;
        S.sv[c] = Vc;
    } else {
        S.se[c] += e;
        S.su[c] += Uc;
        S.sv[c] += Vc;
    }
}

__global__ __launch_bounds__(BX * BY) void k_baro_uv(const DevState S, const double dtau, const int last) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= S.nx || j >= S.ny) return;
    const long long c = idx2(S, i, j);
    const double e = S.eta[c];
    const double hu = S.hu[c], hv = S.hv[c];
    const double Un = hu > 0.0 ? S.ubt[c] + dtau * (-S.g * hu * (e - S.eta[c - 1]) / S.dxc[j] + S.gU[c]) : 0.0;
    const double Vn = hv > 0.0 ? S.vbt[c] + dtau * (-S.g * hv * (e - S.eta[c - S.p2]) / S.dy + S.gV[c]) : 0.0;
    S.ubt[c] = Un;
    S.vbt[c] = Vn;
    wrap2(S, S.ubt, i, j, Un);
    wrap2(S, S.vbt, i, j, Vn);
    if (last) {
        const double ns = double(S.n_substeps);
        S.eta_mean[c] = S.se[c] / ns;
        S.ubt_mean[c] = S.su[c] / ns;
        S.vbt_mean[c] = S.sv[c] / ns;
    }
}

hipError_t launch_barotropic(const DevState& s, hipStream_t st) {
    dim3 block(BX, BY);
    dim3 grid((s.nx + BX - 1) / BX, (s.ny + BY - 1) / BY);
    const double dtau = s.dt / s.n_substeps;
    for (int m = 0; m < s.n_substeps; ++m) {
        hipLaunchKernelGGL(k_baro_eta, grid, block, 0, st, s, dtau, m);
        hipLaunchKernelGGL(k_baro_uv, grid, block, 0, st, s, dtau, (int)(m == s.n_substeps - 1));
    }
    return hipGetLastError();
}

}  // namespace ocn
