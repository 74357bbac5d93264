// k_baro.hip -- the sub-cycled barotropic free-surface loop (paper Sec. 5.3).
//
// Forward-backward substeps in FP64 for every precision: the free surface
// first, from the divergence of the depth-integrated transports, then the
// transports from the new surface gradient plus the slow forcing left by the
// tendency kernel. The substeps run on to t^n + 3dt/2 (M = Ns + Ns/2 of them).
// The new eta, U, V are averages of the substep values with weights a_q
// centred on t^{n+1} (cos^2 window of half-width dt/2, a table on the device);
// the transport that moved the free surface over the step, used for the
// baroclinic correction, is Ubar = sum_l A_l U^l / Ns with A_l = sum_{q>l} a_q.
// The one-substep path takes two launches per substep (surface, then
// transports), every thread updating one column in place and writing the
// periodic copies of its value into the halo the next launch reads.
#include "ocn_dev.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

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
    const double Am = S.baro_A[m], am = S.baro_a[m + 1];
    if (m == 0) {
        S.su[c] = Am * Uc;
        S.sv[c] = Am * Vc;
        S.se[c] = am * e;
    } else {
        S.su[c] += Am * Uc;
        S.sv[c] += Am * Vc;
        S.se[c] += am * e;
    }
}

__global__ __launch_bounds__(BX * BY) void k_baro_uv(const DevState S, const double dtau, const int m) {
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
    const double am = S.baro_a[m + 1];
    S.sfu[c] = (m == 0) ? am * Un : S.sfu[c] + am * Un;
    S.sfv[c] = (m == 0) ? am * Vn : S.sfv[c] + am * Vn;
}

// After the last substep of the one-substep path: the window averages become
// the new state (a launch of its own, since neighbours read eta in k_baro_uv).
__global__ __launch_bounds__(BX * BY) void k_baro_finish(const DevState S) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= S.nx || j >= S.ny) return;
    const long long c = idx2(S, i, j);
    const double ns = double(S.n_substeps);
    const double e = S.se[c], U = S.sfu[c], V = S.sfv[c];
    S.eta[c] = e;
    S.ubt[c] = U;
    S.vbt[c] = V;
    wrap2(S, S.eta, i, j, e);
    wrap2(S, S.ubt, i, j, U);
    wrap2(S, S.vbt, i, j, V);
    S.eta_mean[c] = e;
    S.ubt_mean[c] = S.su[c] / ns;
    S.vbt_mean[c] = S.sv[c] / ns;
}

hipError_t launch_barotropic_fused(const DevState& s, hipStream_t st);

hipError_t launch_barotropic(const DevState& s, hipStream_t st) {
    if (s.baro_fuse >= 2) return launch_barotropic_fused(s, st);
    dim3 block(BX, BY);
    dim3 grid((s.nx + BX - 1) / BX, (s.ny + BY - 1) / BY);
    const double dtau = s.dt / s.n_substeps;
    for (int m = 0; m < s.baro_m; ++m) {
        hipLaunchKernelGGL(k_baro_eta, grid, block, 0, st, s, dtau, m);
        hipLaunchKernelGGL(k_baro_uv, grid, block, 0, st, s, dtau, m);
    }
    hipLaunchKernelGGL(k_baro_finish, grid, block, 0, st, s);
    return hipGetLastError();
}

}  // namespace ocn

namespace ocn {

// Temporally blocked substeps: one launch advances SH substeps of a 64 x 32
// (or, on small grids, 32 x 16) tile held in LDS with an SH-wide halo (the
// halo width is a template parameter, so the LDS of a launch is sized to its
// substep count). Each substep the region of correct values shrinks by one
// cell on every side, so after SH substeps the tile interior is exact; the
// halo cells are recomputed redundantly instead of exchanged. Every point
// carries the same arithmetic as the one-substep path. A tile's halo is its
// neighbours' interior, which they overwrite during the same launch, so
// launches read one buffer of eta, U, V and write the other (parity selects
// which); after an odd number of launches a copy kernel returns the result to
// the primary buffers.
//
// Within a substep each thread updates its own points in place: the surface
// update reads a point's own eta and its neighbours' transports, the
// transport update its own transports and its neighbours' eta, so two
// barriers per substep suffice (after each update). The window sums of the
// interior points read eta after the first barrier and U, V after the
// second, while no thread writes them.
constexpr int FSMAX = 8, FT = 512;
// Tile shapes: kBaroTileX x kBaroTileY for large grids and the ensembles;
// 32 x 16 where that costs less (use_small_tiles): small tiles recompute more
// halo per interior point but fill the last round of workgroups better.
constexpr int kSmallTileX = 32, kSmallTileY = 16;


// Registers hold only what each halo-inclusive point needs every substep
// (depths and slow forcing); row metrics sit in small LDS tables, and the
// window sums live with a second mapping over the interior points only (FI
// per thread). The depths of a point's u and v columns are looked up from
// their wet-layer counts (one 4-byte count per point instead of two 8-byte
// depths from memory). Window flags: bit 0, the sums of the averaging window
// carried in are not all zero (read them); bit 1, they are not all zero after
// this launch (write them); launches before the window's first nonzero weight
// skip both.
template <int BX, int BY, int SH>
__device__ __forceinline__ void baro_tile(const DevState& S, const int bx, const int by, const double dtau,
                                          const int m0, const int first, const int last, const int parity,
                                          const int wflags) {
    constexpr int FBX = BX, FBY = BY;
    constexpr int FEW = FBX + 2 * SH, FEH = FBY + 2 * SH, FEN = FEW * FEH;
    constexpr int FQ = (FEN + FT - 1) / FT;  // halo-inclusive points per thread
    constexpr int FI = FBX * FBY / FT;       // interior points per thread
    static_assert(FBX * FBY % FT == 0, "interior points must divide evenly over the threads");
    // state tiles with a row of padding before and after, so that the
    // neighbours e +- 1 and e +- FEW of every point are addresses of the tile
    // (values there are garbage by the halo argument and never reach the
    // interior)
    __shared__ double sEp[FEN + 2 * FEW], sUp[FEN + 2 * FEW], sVp[FEN + 2 * FEW];
    double* const sE = sEp + FEW;
    double* const sU = sUp + FEW;
    double* const sV = sVp + FEW;
    // per-row coefficients of the surface update (dtau/A times dy, dxv south,
    // dxv north) and of the zonal transport update (-g dtau / dxc)
    __shared__ double sCdy[FEH], sC0[FEH], sC1[FEH], sCu[FEH];
    __shared__ double sCum[kMaxLevels + 1];
    __shared__ double sWa[SH], sWA[SH];  // a_{m0+1+m} and A_{m0+m} of the launch's substeps
    const double* __restrict__ inE = parity ? S.eta2 : S.eta;
    const double* __restrict__ inU = parity ? S.ubt2 : S.ubt;
    const double* __restrict__ inV = parity ? S.vbt2 : S.vbt;
    double* __restrict__ outE = parity ? S.eta : S.eta2;
    double* __restrict__ outU = parity ? S.ubt : S.ubt2;
    double* __restrict__ outV = parity ? S.vbt : S.vbt2;
    const int tid = threadIdx.x;
    const int i0 = bx * FBX, j0 = by * FBY;
    const int nx = S.nx, ny = S.ny;
    const double dy = S.dy, g = S.g;

    for (int k = tid; k <= S.nz; k += FT) sCum[k] = S.cumh[k];
    if (tid < SH) {
        sWa[tid] = S.baro_a[m0 + tid + 1];
        sWA[tid] = S.baro_A[m0 + tid];
    }
    // row metrics (rows past a closed edge take the nearest row; unused)
    for (int lj = tid; lj < FEH; lj += FT) {
        int gj = j0 - SH + lj;
        if (S.periodic_y) gj = ((gj % ny) + ny) % ny;
        const int jm = min(max(gj, 0), ny - 1);
        const double ra = dtau / S.area[jm];
        sCdy[lj] = ra * S.dy;
        sC0[lj] = ra * S.dxv[jm];
        sC1[lj] = ra * S.dxv[jm + 1];
        sCu[lj] = -S.g * dtau / S.dxc[jm];
    }
    for (int q = tid; q < FEW; q += FT) {
        sEp[q] = 0.0; sUp[q] = 0.0; sVp[q] = 0.0;
        sEp[FEN + FEW + q] = 0.0; sUp[FEN + FEW + q] = 0.0; sVp[FEN + FEW + q] = 0.0;
    }
    // halo-inclusive points: forcing and wet-layer counts of the u and v
    // columns, and the state into LDS. Every load is issued (at a valid,
    // clamped address) before any is used, so that the waits for them do not
    // serialise the points. The transport update of a point is
    // U + Cu (eta - eta_west) + Gu with Cu = -g dtau Hu / dxc and Gu = dtau gU
    // (V likewise with dy), Cu = 0 on dry faces.
    double gU[FQ], gV[FQ], Hu[FQ], Hv[FQ];
    int Ku[FQ], Kv[FQ];
    double aU[FI], aV[FI];          // interior points: sum_l A_l U^l, V^l (transport of the step)
    double fE[FI], fU[FI], fV[FI];  // sum_q a_q eta^q, U^q, V^q (new state)
    int ie[FI];                     // LDS index, -1 outside the domain
    {
        double lE[FQ], lU[FQ], lV[FQ];
        int kc[FQ], kw[FQ], ks[FQ];
        bool in[FQ];
#pragma unroll
        for (int q = 0; q < FQ; ++q) {
            const int e = tid + q * FT;
            const int li = e % FEW, lj = e / FEW;
            int gi = i0 - SH + li, gj = j0 - SH + lj;
            bool inside = e < FEN;
            if (S.periodic_x) gi = ((gi % nx) + nx) % nx;
            else inside = inside && gi >= 0 && gi < nx;
            if (S.periodic_y) gj = ((gj % ny) + ny) % ny;
            else inside = inside && gj >= 0 && gj < ny;
            const int gic = inside ? gi : 0, jmc = inside ? min(max(gj, 0), ny - 1) : 0;
            const long long c = idx2(S, gic, jmc);
            in[q] = inside;
            gU[q] = S.gU[c];
            gV[q] = S.gV[c];
            lE[q] = inE[c];
            lU[q] = inU[c];
            lV[q] = inV[c];
            kc[q] = S.kb[idxk(S, gic, jmc)];
            kw[q] = S.kb[idxk(S, gic - 1, jmc)];
            ks[q] = S.kb[idxk(S, gic, jmc - 1)];
        }
        // interior points: window sums carried between launches (issued with
        // the point loads)
#pragma unroll
        for (int p = 0; p < FI; ++p) {
            const int pp = tid + p * FT;
            const int ti = i0 + pp % FBX, tj = j0 + pp / FBX;
            const bool live = ti < nx && tj < ny;
            ie[p] = live ? (SH + pp / FBX) * FEW + SH + pp % FBX : -1;
            const long long c = idx2(S, live ? ti : 0, live ? tj : 0);
            const bool carry = live && !first;
            const bool carryw = carry && (wflags & 1);
            aU[p] = carry ? S.su[c] : 0.0;
            aV[p] = carry ? S.sv[c] : 0.0;
            fE[p] = 0.0;
            fU[p] = 0.0;
            fV[p] = 0.0;
            if (carryw) {
                fE[p] = S.se[c];
                fU[p] = S.sfu[c];
                fV[p] = S.sfv[c];
            }
        }
#pragma unroll
        for (int q = 0; q < FQ; ++q) {
            const int e = tid + q * FT;
            const bool inside = in[q];
            gU[q] = inside ? gU[q] : 0.0;
            gV[q] = inside ? gV[q] : 0.0;
            Ku[q] = inside ? min(kc[q], kw[q]) : 0;
            Kv[q] = inside ? min(kc[q], ks[q]) : 0;
            if (e < FEN) {
                sE[e] = inside ? lE[q] : 0.0;
                sU[e] = inside ? lU[q] : 0.0;
                sV[e] = inside ? lV[q] : 0.0;
            }
        }
    }
    __syncthreads();
    {
        const double cv = -g * dtau / dy;
#pragma unroll
        for (int q = 0; q < FQ; ++q) {
            const int lj = min((tid + q * FT) / FEW, FEH - 1);
            Hu[q] = sCum[Ku[q]] * sCu[lj];
            Hv[q] = sCum[Kv[q]] * cv;
            gU[q] *= dtau;
            gV[q] *= dtau;
        }
    }
    // the transport sum takes U^l at the start of each substep l
    {
        const double A0 = sWA[0];
#pragma unroll
        for (int p = 0; p < FI; ++p) {
            if (ie[p] < 0) continue;
            aU[p] += A0 * sU[ie[p]];
            aV[p] += A0 * sV[ie[p]];
        }
    }

    int tq = tid;
    for (int m = 0; m < SH; ++m) {
        // each point's LDS neighbours are recomputed from the thread index every
        // substep (a few integer operations) rather than kept in registers
        asm volatile("" : "+v"(tq));
        const double am = sWa[m];
        // Rows that matter at substep m: below row m the transports and
        // above row FEH-2-m the surface are already invalid (the region of
        // correct values shrinks by a row on each side per substep, as
        // eta(r) reads V(r), V(r+1) and V(r) reads eta(r-1), eta(r)), so only
        // rows m .. FEH-2-m are updated; whole waves outside skip the work.
        const int rlo = m, rhi = FEH - 2 - m;
        // free surface from the divergence of the transports, in place
#pragma unroll
        for (int q = 0; q < FQ; ++q) {
            const int e = tq + q * FT;
            const int lj = e / FEW;
            if (e < FEN && lj >= rlo && lj <= rhi) {
                const double div = sCdy[lj] * (sU[e + 1] - sU[e]) + sC1[lj] * sV[e + FEW] - sC0[lj] * sV[e];
                sE[e] = sE[e] - div;
            }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < FI; ++p) {
            if (ie[p] < 0) continue;
            fE[p] += am * sE[ie[p]];
        }
        // transports from the new surface slope plus the slow forcing, in place
#pragma unroll
        for (int q = 0; q < FQ; ++q) {
            const int e = tq + q * FT;
            const int lj = e / FEW;
            if (e < FEN && lj >= rlo && lj <= rhi) {
                const double ec = sE[e];
                const double un = Hu[q] != 0.0 ? sU[e] + fma(Hu[q], ec - sE[e - 1], gU[q]) : 0.0;
                const double vn = Hv[q] != 0.0 ? sV[e] + fma(Hv[q], ec - sE[e - FEW], gV[q]) : 0.0;
                sU[e] = un;
                sV[e] = vn;
            }
        }
        __syncthreads();
        const double An = (m + 1 < SH) ? sWA[m + 1 < SH ? m + 1 : 0] : 0.0;
#pragma unroll
        for (int p = 0; p < FI; ++p) {
            if (ie[p] < 0) continue;
            const double u = sU[ie[p]], v = sV[ie[p]];
            fU[p] += am * u;
            fV[p] += am * v;
            if (m + 1 < SH) {
                aU[p] += An * u;
                aV[p] += An * v;
            }
        }
    }

    // write the interior (with its periodic halo copies): the instantaneous
    // state between launches, the window averages after the last one
#pragma unroll
    for (int p = 0; p < FI; ++p) {
        if (ie[p] < 0) continue;
        const int pp = tid + p * FT;
        const int gi = i0 + pp % FBX, gj = j0 + pp / FBX;
        const long long c = idx2(S, gi, gj);
        const int e = ie[p];
        const double vE = last ? fE[p] : sE[e];
        const double vU = last ? fU[p] : sU[e];
        const double vV = last ? fV[p] : sV[e];
        outE[c] = vE;
        outU[c] = vU;
        outV[c] = vV;
        for_each_image(S, gi, gj, S.h, [&](int x, int y) {
            const long long o = idx2(S, x, y);
            outE[o] = vE;
            outU[o] = vU;
            outV[o] = vV;
        });
        if (last) {
            const double ns = double(S.n_substeps);
            S.eta_mean[c] = fE[p];
            S.ubt_mean[c] = aU[p] / ns;
            S.vbt_mean[c] = aV[p] / ns;
        } else {
            S.su[c] = aU[p];
            S.sv[c] = aV[p];
            if (wflags & 2) {
                S.se[c] = fE[p];
                S.sfu[c] = fU[p];
                S.sfv[c] = fV[p];
            }
        }
    }
}

// Occupancy target: two 8-wave workgroups per CU while their LDS fits (halo
// widths up to 7 on 64 x 24 tiles), else one.
template <int BX, int BY, int SH> struct BaroWaves {
    static constexpr int n = ((BX + 2 * SH) * (BY + 2 * SH) + 2 * (BX + 2 * SH)) * 24 <= 78 * 1024 ? 4 : 2;
};

template <int BX, int BY, int SH>
__global__ __launch_bounds__(FT) __attribute__((amdgpu_waves_per_eu(BaroWaves<BX, BY, SH>::n))) void k_baro_fused(
    const DevState S, const double dtau, const int m0, const int first, const int last, const int parity,
    const int wflags, const int gx) {
    // row-major tiles in per-XCD ranges (halo rows of a tile come from the L2
    // its neighbours filled)
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    baro_tile<BX, BY, SH>(S, t % gx, t / gx, dtau, m0, first, last, parity, wflags);
}

// Second buffers back to the primary ones (whole padded arrays, halos included).
__global__ __launch_bounds__(256) void k_baro_copyback(const DevState S) {
    const long long o2 = (long long)S.h * S.p2 + S.ox2;
    const long long n = (long long)S.p2 * (S.ny + 2 * S.h);
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    (S.eta - o2)[e] = (S.eta2 - o2)[e];
    (S.ubt - o2)[e] = (S.ubt2 - o2)[e];
    (S.vbt - o2)[e] = (S.vbt2 - o2)[e];
}

__global__ __launch_bounds__(256) void k_baro_copyback_batched(const DevState* __restrict__ members, const int m0) {
    const DevState& S = members[m0 + blockIdx.y];
    const long long o2 = (long long)S.h * S.p2 + S.ox2;
    const long long n = (long long)S.p2 * (S.ny + 2 * S.h);
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        (S.eta - o2)[e] = (S.eta2 - o2)[e];
        (S.ubt - o2)[e] = (S.ubt2 - o2)[e];
        (S.vbt - o2)[e] = (S.vbt2 - o2)[e];
    }
}

// Ensemble: entry blockIdx.x of the table is (member, bx, by).
template <int SH>
__global__ __launch_bounds__(FT) __attribute__((amdgpu_waves_per_eu(BaroWaves<kBaroTileX, kBaroTileY, SH>::n))) void k_baro_fused_batched(const DevState* __restrict__ members,
                                                           const int4* __restrict__ tiles, const double dtau,
                                                           const int m0, const int first, const int last,
                                                           const int parity, const int wflags) {
    const int4 e = tiles[blockIdx.x];
    baro_tile<kBaroTileX, kBaroTileY, SH>(members[e.x], e.y, e.z, dtau, m0, first, last, parity, wflags);
}

// The same over a queue of table entries, with persistent workgroups.
template <int SH>
__global__ __launch_bounds__(FT) __attribute__((amdgpu_waves_per_eu(BaroWaves<kBaroTileX, kBaroTileY, SH>::n))) void k_baro_fused_queued(const DevState* __restrict__ members,
                                                           const int4* __restrict__ tiles, const int ntiles,
                                                           const double dtau, const int m0, const int first,
                                                           const int last, const int parity, const int wflags,
                                                           int* __restrict__ queue) {
    for_each_queued_tile(queue, ntiles, [&](int b) {
        const int4 e = tiles[b];
        baro_tile<kBaroTileX, kBaroTileY, SH>(members[e.x], e.y, e.z, dtau, m0, first, last, parity, wflags);
    });
}

__global__ __launch_bounds__(256) void k_zero_counters(int* p, const int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_zero_counters(int* p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_counters, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

// Instantiations per halo width 1..FSMAX: f<SH>() launches the kernel of that width.
template <class F>
hipError_t by_halo(int s, F&& f) {
    switch (s) {
    case 1: return f(std::integral_constant<int, 1>());
    case 2: return f(std::integral_constant<int, 2>());
    case 3: return f(std::integral_constant<int, 3>());
    case 4: return f(std::integral_constant<int, 4>());
    case 5: return f(std::integral_constant<int, 5>());
    case 6: return f(std::integral_constant<int, 6>());
    case 7: return f(std::integral_constant<int, 7>());
    case 8: return f(std::integral_constant<int, 8>());
    default: return hipErrorInvalidValue;
    }
}

int baro_substeps(int n_substeps) { return n_substeps + n_substeps / 2; }

// Workgroups of a kernel that fit on the current device at once (cached per
// kernel and device).
int resident_workgroups(const void* kernel, int block_threads) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({kernel, dev});
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block_threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    const int n = per_cu * cus;
    cache[{kernel, dev}] = n;
    return n;
}

// First substep q (1-based) whose window weight a_q is nonzero: the weights
// are cos^2(pi t), t = q/Ns - 1, on |t| < 1/2 (the same test as the table's).
static int window_first(int n_substeps) {
    const int M = baro_substeps(n_substeps);
    for (int q = 1; q <= M; ++q)
        if (std::fabs(double(q) / n_substeps - 1.0) < 0.5) return q;
    return M + 1;
}

// Window flags of a launch running substeps m0 .. m0+ss-1 (weights a_{m0+1} ..
// a_{m0+ss}): read the carried sums if a weight before m0+1 was nonzero, write
// them if one up to m0+ss was.
static int window_flags(int n_substeps, int m0, int ss) {
    const int qf = window_first(n_substeps);
    return (m0 >= qf ? 1 : 0) | (m0 + ss >= qf ? 2 : 0);
}

int baro_launches(int n_substeps, int fuse) {
    const int sub = std::max(2, std::min(fuse, FSMAX));
    const int M = baro_substeps(n_substeps);
    return (M + sub - 1) / sub;
}

hipError_t launch_barotropic_batched(const DevState* members, int n_members, const int4* tiles, int ntiles,
                                     int n_substeps, int fuse, double dt, int* queue, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    const int sub = std::max(2, std::min(fuse, FSMAX));
    const double dtau = dt / n_substeps;
    const int M = baro_substeps(n_substeps);
    int parity = 0, group = 0;
    for (int m0 = 0; m0 < M; m0 += sub, parity ^= 1, ++group) {
        const int ss = std::min(sub, M - m0);
        const int first = m0 == 0, last = m0 + ss == M;
        const int wf = window_flags(n_substeps, m0, ss);
        hipError_t e = by_halo(ss, [&](auto h) {
            constexpr int SH = decltype(h)::value;
            if (queue) {
                const int nb = std::min(ntiles, resident_workgroups((const void*)k_baro_fused_queued<SH>, FT));
                hipLaunchKernelGGL((k_baro_fused_queued<SH>), dim3(nb), dim3(FT), 0, st, members, tiles, ntiles, dtau,
                                   m0, first, last, parity, wf, queue + 8 * group);
            } else {
                hipLaunchKernelGGL((k_baro_fused_batched<SH>), dim3(ntiles), dim3(FT), 0, st, members, tiles, dtau,
                                   m0, first, last, parity, wf);
            }
            return hipSuccess;
        });
        if (e != hipSuccess) return e;
    }
    if (parity) {  // the result sits in the second buffers
        for (int m0 = 0; m0 < n_members; m0 += 65535)
            hipLaunchKernelGGL(k_baro_copyback_batched, dim3(64, std::min(65535, n_members - m0)), dim3(256), 0, st,
                               members, m0);
    }
    return hipGetLastError();
}

// Small tiles recompute more halo per interior point: (32 + 2s)(16 + 2s) /
// 512 against (64 + 2s)(24 + 2s) / 1536, 1.40 times as many points at s = 7.
// They pay where the large tiles leave the device idle: a launch runs
// ceil(tiles / resident) rounds of workgroups, and the large tiles fill the
// fraction tiles / (rounds x resident) of them. Small tiles are taken when
// that fill times the halo ratio is below 1. At 1/4 degree (1440 x 600) the
// 575 large tiles fill 0.56 of two rounds and the small tiles cost less
// (0.56 against 0.66 ms per step); at 1/12 degree the 5100 large tiles fill
// ten rounds and win (small tiles there took 4.06 against 3.86 ms).
static bool use_small_tiles(const DevState& s, int sub) {
    const long long n = (long long)((s.nx + kBaroTileX - 1) / kBaroTileX) * ((s.ny + kBaroTileY - 1) / kBaroTileY);
    const long long slots =
        std::max(1, resident_workgroups((const void*)k_baro_fused<kBaroTileX, kBaroTileY, kBaroFuseDefault>, FT));
    const double fill = double(n) / double(((n + slots - 1) / slots) * slots);
    const double halo = (double((kSmallTileX + 2 * sub) * (kSmallTileY + 2 * sub)) / (kSmallTileX * kSmallTileY)) /
                        (double((kBaroTileX + 2 * sub) * (kBaroTileY + 2 * sub)) / (kBaroTileX * kBaroTileY));
    return fill * halo < 1.0;
}

hipError_t launch_barotropic_fused(const DevState& s, hipStream_t st) {
    const int sub = std::min(s.baro_fuse, FSMAX);
    const bool small = use_small_tiles(s, sub);
    const int bx = small ? kSmallTileX : kBaroTileX, by = small ? kSmallTileY : kBaroTileY;
    const int gx = (s.nx + bx - 1) / bx, gy = (s.ny + by - 1) / by;
    const dim3 grid(gx * gy);
    const double dtau = s.dt / s.n_substeps;
    const int M = s.baro_m;
    int parity = 0;
    for (int m0 = 0; m0 < M; m0 += sub, parity ^= 1) {
        const int ss = std::min(sub, M - m0);
        const int first = m0 == 0, last = m0 + ss == M;
        hipError_t e = by_halo(ss, [&](auto h) {
            constexpr int SH = decltype(h)::value;
            const int wf = window_flags(s.n_substeps, m0, ss);
            if (small)
                hipLaunchKernelGGL((k_baro_fused<kSmallTileX, kSmallTileY, SH>), grid, dim3(FT), 0, st, s, dtau, m0,
                                   first, last, parity, wf, gx);
            else
                hipLaunchKernelGGL((k_baro_fused<kBaroTileX, kBaroTileY, SH>), grid, dim3(FT), 0, st, s, dtau, m0,
                                   first, last, parity, wf, gx);
            return hipSuccess;
        });
        if (e != hipSuccess) return e;
    }
    if (parity) {  // the result sits in the second buffers
        const long long n = (long long)s.p2 * (s.ny + 2 * s.h);
        hipLaunchKernelGGL(k_baro_copyback, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s);
    }
    return hipGetLastError();
}

}  // namespace ocn
