// k_tend.hip -- fused tendency + AB2 predictor kernel.
//
// One kernel computes, for every wet cell of a level, the three tendencies of
// the baroclinic step (paper Sec. 5.1: one fused tendency computation per
// prognostic variable, with hydrostatic pressure as the only 3D diagnostic,
// here integrated in registers instead of stored): flux-form WENO advection of
// T, u and v, energy-conserving Coriolis with the spherical metric term, the
// hydrostatic pressure gradient of a linear equation of state, wind stress and
// surface restoring in the top layer; then the AB2 predictor (paper Sec. 5.2)
// phi* = phi + dt ((3/2+chi) G^n - (1/2+chi) G^{n-1}), and the depth integral
// of the AB2 momentum tendency that forces the barotropic mode.
//
// Mapping. A TX x TY workgroup (32 x 16 in FP32, 16 x 16 in FP64; the
// batched ensemble kernel uses 64 x 4 or 64 x 8) owns a tile of
// (TX-1) x (TY-1) columns and marches from the surface to the bottom. Tiles are
// handed out so that the eight XCDs each sweep a contiguous band of the grid:
// neighbouring tiles share an L2 and, marching in near lockstep, reuse each
// other's halo rows from it. Thread (tx, ty) sits on point
// (i0 - 1 + tx, j0 - 1 + ty); at each level it computes, into LDS, the quantities
// that live at its point: the T flux through the east and north faces, the u
// flux through the cell centre and the north-west corner, the v flux through
// the south-east corner and the cell centre, Q v_c and Q u_c (Coriolis), the
// pressure and the vertical transport of its column. Every face flux is
// therefore computed once, and a cell reads its west/south fluxes from the
// neighbouring thread: conservation holds to round-off. The first row and
// column of threads only supply these neighbour values.
//
// Vertical structure. Pressure integrates downward from p = 0 at the surface;
// the vertical transport W integrates downward from its surface value
// W(top) = -(divergence of the depth-integrated transport), computed from the
// column sums of u and v left by the previous column kernel, so that both run
// in the same top-down march. The own column's values at six levels (k+2 ..
// k-3) stay in registers for the vertical WENO stencils.
//
// Temperature is stored as T' = T - tref(k). Horizontal reconstructions of T'
// equal those of T minus tref (WENO is invariant under adding a constant); the
// vertical ones reconstruct T from stencil differences that include the tref
// steps, and the advection of the reference profile is added back in exact
// algebraic form. In FP32 this keeps the 0.01 K noise that drives the pressure
// gradient free of the cancellation a 20 K absolute temperature would cause.
#include "ocn_dev.h"

#include <algorithm>

namespace ocn {

constexpr int TXB = 64;  // tile width of the batched ensemble launches (the host builds 63-column tiles)

// Workgroup shape of the single-state launch: TX x TY threads own
// (TX - 1) x (TY - 1) columns, so the ring of threads that only supply
// neighbour fluxes costs TX TY / ((TX - 1)(TY - 1)) - 1 extra work.
template <typename R> struct TendShape;
template <> struct TendShape<float> { static constexpr int TX = 32, TY = 16; };
template <> struct TendShape<double> { static constexpr int TX = 16, TY = 16; };
template <typename R> struct TendShapeSalt { static constexpr int TX = TendShape<R>::TX, TY = TendShape<R>::TY; };
template <> struct TendShapeSalt<float> { static constexpr int TX = 32, TY = 8; };

template <typename R> struct Eps;
template <> struct Eps<double> { static constexpr double v = 1e-8; };
template <> struct Eps<float> { static constexpr float v = 1e-8f; };

// Reciprocals: the hardware estimate in FP32 (1 ulp); in FP64 the estimate
// refined by two Newton steps.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

// 1/dz of a level: the FP64 quotient in FP64, the hardware reciprocal of the
// rounded thickness in FP32 (a level value that every lane would otherwise
// divide in FP64).
__device__ __forceinline__ double inv_level(double dz, double) { return 1.0 / dz; }
__device__ __forceinline__ float inv_level(double dz, float) { return __builtin_amdgcn_rcpf(float(dz)); }

// Fifth-order WENO-Z face value (Borges et al. 2008) on Jiang-Shu smoothness
// indicators; c is the upwind cell, the face lies between c and d. Written in
// the differences d1..d4 of neighbouring values, with exact rescalings that
// save instructions:
//  - the indicators and eps are taken 4 times larger, beta'_k = 13/3 s_k^2 +
//    r_k^2 with s the second and r the first difference of stencil k; the
//    WENO-Z ratios tau / (beta_k + eps) are unchanged, and the three share
//    one reciprocal of the product of their denominators (all >= 4 eps);
//    eps enters each indicator inside its fused multiply-adds, and
//    tau = |beta_0 - beta_2| is taken from the sums with eps (it cancels);
//  - with w_k = 1 + (tau / (beta_k + eps))^2 the nonlinear weights are
//    d_k w_k (d = 1/10, 6/10, 3/10), so d_k is folded into the candidate
//    values: c + sum w_k (d_k q_k) / sum d_k w_k, where q_k - c is the
//    quadratic candidate of stencil k as a combination of differences.
template <typename R>
__device__ __forceinline__ R weno5z(R a, R b, R c, R d, R e) {
    const R d1 = b - a, d2 = c - b, d3 = d - c, d4 = e - d;
    const R s0 = d2 - d1, s1 = d3 - d2, s2 = d4 - d3;          // second differences
    const R r0 = fma(R(2), d2, s0), r1 = d2 + d3, r2 = fma(R(-2), d3, s2);
    const R k13 = R(13) / R(3), eps4 = R(4) * Eps<R>::v;
    const R e0 = fma(s0 * s0, k13, fma(r0, r0, eps4));  // beta'_k + eps
    const R e1 = fma(s1 * s1, k13, fma(r1, r1, eps4));
    const R e2 = fma(s2 * s2, k13, fma(r2, r2, eps4));
    const R tau = fabs(e0 - e2);
    const R p12 = e1 * e2, p02 = e0 * e2, p01 = e0 * e1;
    const R tr = tau * rcp(p01 * e2);
    const R z0 = tr * p12, z1 = tr * p02, z2 = tr * p01;
    const R w0 = fma(z0, z0, R(1)), w1 = fma(z1, z1, R(1)), w2 = fma(z2, z2, R(1));
    // d_k (q_k - c): (5 d2 - 2 d1)/60, (d2 + 2 d3)/10, (4 d3 - d4)/20
    const R q0 = fma(R(1.0 / 12.0), d2, R(-1.0 / 30.0) * d1);
    const R q1 = fma(R(0.2), d3, R(0.1) * d2);
    const R q2 = fma(R(0.2), d3, R(-0.05) * d4);
    const R den = fma(R(0.1), w0, fma(R(0.6), w1, R(0.3) * w2));
    return c + fma(w0, q0, fma(w1, q1, w2 * q2)) * rcp(den);
}

// Third-order WENO-JS face value on (b, c, d), c upwind.
template <typename R>
__device__ __forceinline__ R weno3(R b, R c, R d) {
    const R q0 = R(0.5) * (R(3) * c - b);
    const R q1 = R(0.5) * (c + d);
    const R e0 = (c - b) * (c - b) + Eps<R>::v;
    const R e1 = (d - c) * (d - c) + Eps<R>::v;
    const R a0 = (R(1) / R(3)) * rcp(e0 * e0);
    const R a1 = (R(2) / R(3)) * rcp(e1 * e1);
    return (a0 * q0 + a1 * q1) * rcp(a0 + a1);
}

// Order-adaptive reconstruction: WENO5 when all five points are valid, WENO3
// when the three central ones are, else the upwind value.
template <typename R>
__device__ __forceinline__ R recon(R a, R b, R c, R d, R e, bool oa, bool ob, bool oc, bool od, bool oe) {
    if (oa && ob && oc && od && oe) return weno5z(a, b, c, d, e);
    if (ob && oc && od) return weno3(b, c, d);
    return c;
}

// Flux F * phi_face through a face with the six values p0..p5 at points -3..+2
// around it (face between points -1 and 0); ok flags each point.
template <typename R>
__device__ __forceinline__ R upwind_flux(R F, const R* p, const bool* ok) {
    if (F == R(0)) return R(0);
    const bool pos = F > R(0);
    const R a = pos ? p[0] : p[5], b = pos ? p[1] : p[4], c = pos ? p[2] : p[3];
    const R d = pos ? p[3] : p[2], e = pos ? p[4] : p[1];
    const bool oa = pos ? ok[0] : ok[5], ob = pos ? ok[1] : ok[4], oc = pos ? ok[2] : ok[3];
    const bool od = pos ? ok[3] : ok[2], oe = pos ? ok[4] : ok[1];
    return F * recon(a, b, c, d, e, oa, ob, oc, od, oe);
}

// Same with all six points valid (the open-ocean case).
template <typename R>
__device__ __forceinline__ R upwind_flux_wet(R F, const R* p) {
    const bool pos = F > R(0);
    const R a = pos ? p[0] : p[5], b = pos ? p[1] : p[4], c = pos ? p[2] : p[3];
    const R d = pos ? p[3] : p[2], e = pos ? p[4] : p[1];
    return F * weno5z(a, b, c, d, e);
}

// The reconstructed value (not the flux) at the point between p2 and p3,
// upwind of F (the right-biased stencil when F <= 0), all six points valid
// or with validity flags.
template <typename R>
__device__ __forceinline__ R upwind_value_wet(R F, const R* p) {
    const bool pos = F > R(0);
    return weno5z(pos ? p[0] : p[5], pos ? p[1] : p[4], pos ? p[2] : p[3], pos ? p[3] : p[2], pos ? p[4] : p[1]);
}
template <typename R>
__device__ __forceinline__ R upwind_value(R F, const R* p, const bool* ok) {
    const bool pos = F > R(0);
    return recon(pos ? p[0] : p[5], pos ? p[1] : p[4], pos ? p[2] : p[3], pos ? p[3] : p[2], pos ? p[4] : p[1],
                 pos ? ok[0] : ok[5], pos ? ok[1] : ok[4], pos ? ok[2] : ok[3], pos ? ok[3] : ok[2],
                 pos ? ok[4] : ok[1]);
}

// Vorticity is reconstructed in units of a typical Coriolis parameter (1/s),
// so that WENO's absolute epsilon sits below the smoothness indicators of
// ocean vorticity as it does for order-one data.
constexpr double kZetaRef = 1e-4;

// The tile order: bands of kTendBand tile rows, each walked column by column
// (down the band, then one column east), so that some of the north and south
// halo rows of the tiles an XCD runs at once are read from its L2 by the
// tile above or below. Measured at 1/12 degree (FP32, 32 x 16 tiles): bands
// of 2 rows fetch 56.1 GB from memory per launch against 57.5 for the plain
// row-major order (1 % faster); bands of 4 and 8 fetch 58.3 and 65.0 and run
// slower, as the square blocks give up the sharing of partial cache lines
// between east and west neighbours; without the per-XCD ranges the fetch is
// 76.6 GB.
constexpr int kTendBand = 2;
__device__ __forceinline__ int2 band_tile(int t, int gx, int gy) {
    const int per = gx * kTendBand;
    const int b = t / per, r = t - b * per;
    const int h = min(kTendBand, gy - b * kTendBand);  // the last band may be shorter
    return make_int2(r / h, b * kTendBand + r % h);
}

// Occupancy target per precision: four waves per SIMD (two FP32 workgroups of
// 8 waves per CU) keeps the FP32 kernel within 128 VGPRs, and so does the
// vector-invariant momentum form on the same 32 x 16 tiles (11 % faster than
// 32 x 8 tiles at three waves). The second tracer needs about 170 VGPRs in
// FP32: its 32 x 8 tiles run at three waves per SIMD (three 4-wave workgroups
// per CU; 25 % faster than 32 x 16 tiles at two), with or without the
// vector-invariant form. The FP64 salinity kernel on 64 x 4 tiles holds one
// workgroup per CU (two would exceed the LDS).
template <typename R, bool SALT, int TY> struct TendWaves {
    static constexpr int n = (sizeof(R) == 4 && !SALT)            ? 4
                             : (sizeof(R) == 4 && SALT && TY == 8) ? 3
                             : (sizeof(R) == 4 && SALT && TY == 16) ? 4
                             : (sizeof(R) == 8 && SALT && TY == 4) ? 1
                                                                   : 2;
};

// One tile (bx, by) of one state. Called by the single-state kernel and by the
// batched kernel that steps an ensemble of basins in one launch.
//
// Forward-backward pressure. The momentum step takes the hydrostatic pressure
// of T^n + eps dt Ghat_T, the tracer just predicted by AB2 weighted by eps,
// not an extrapolated pressure gradient (AB2 alone amplifies the internal
// gravity waves that converging meridians bring to a frequency times dt near
// 1). The u point on a cell's west face needs that pressure in the column to
// its west, and the v point on its south face in the column to its south, so
// the ring threads (column tx = 0 and row ty = 0) also form the tracer
// tendency of their own column: they read the AB2 history there (it is
// double-buffered, so no tile overwrites a value another still reads) and the
// fluxes through their far faces, which they compute in the flux slots that
// ring threads otherwise leave idle (u through the north-west corner for the
// column, u through the cell centre for the row). Every point's pressure goes
// to LDS; the momentum tendencies of level k are completed one level later,
// when the pressure of level k of the neighbours is in LDS.
//
// Barriers: two per level, after the staging of the level's value tiles and
// after the point quantities. The tiles are double-buffered by level parity,
// so a wave may stage level k-1 while others still read level k; the flux,
// Coriolis and transport arrays of level k are only rewritten after the next
// level's first barrier, which every wave reaches only once it has assembled
// level k; the pressure is double-buffered by parity as well.
//
// Vector-invariant momentum (VI): the momentum flux slots of the cells stay
// idle (the ring keeps using its slots for the tracers); each cell forms
// (f + zeta_hat) vbar for u and -(f + zeta_hat) ubar for v in the point
// phase, zeta_hat reconstructed from corner vorticities that it computes from
// the u, v tiles (six corners along y for u, along x for v); every point puts
// its kinetic energy in LDS for the gradients, and the vertical term is the
// flux form's vertical divergence minus u times the divergence of the
// velocity point's vertical transport.
template <typename R, int TX, int TY, bool SALT, bool VI>
__device__ __forceinline__ void tend_tile(const DevState& S, const int first, const int bx, const int by) {
    constexpr int NT = TX * TY;
    constexpr int LW = TX + 5, LH = TY + 5, LN = LW * LH;  // u, v tiles: points -2 .. +3 around the block
    constexpr int TW = TX + 6, TH = TY + 6, TN = TW * TH;  // T tile: points -3 .. +3
    constexpr int KW = TX + 6, KH = TY + 6, KN = KW * KH;  // wet counts: -3 .. +3
    constexpr int NS = (LN + NT - 1) / NT;                 // u, v tile slots per thread
    constexpr int NST = (TN + NT - 1) / NT;                // T tile slots per thread

    // value tiles, double-buffered by level parity: level k-1 is staged while
    // slower waves may still read level k, so a level needs two barriers
    __shared__ R sT2[2][TN], sU2[2][LN], sV2[2][LN];
    __shared__ int sK[KN];
    __shared__ R fxT[NT], fyT[NT], fxu[NT], fyu[NT], fxv[NT], fyv[NT];
    __shared__ R sQv[NT], sQu[NT], sP[2 * NT], sWm[NT];
    // per-row metrics of the tile's rows (a row's threads read one address):
    // dxv south, dxv north, area, f, tan(phi)/a, 1/area, 1/(dxv dy), 1/dxc
    __shared__ R sRow[9][TY];
    // vector-invariant form: kinetic energy of every point, and the metrics of
    // rows j0-4 .. j0+TY+1 (dxc; 1 / (dxv dy zeta_ref)) for corner vorticities
    constexpr int VNT = VI ? NT : 1, VRR = VI ? TY + 6 : 1;
    __shared__ R sKE[VNT];
    __shared__ R sRX[2][VRR];
    __shared__ R sTop[NT];  // surface volume flux times the full top temperature
    // salinity: its tile, its face fluxes and the surface term, as for T
    constexpr int SN = SALT ? TN : 1, SNT = SALT ? NT : 1;
    __shared__ R sS2[2][SN];
    __shared__ R fxS[SNT], fyS[SNT], sTopS[SNT];
    // Per-level constants, staged once (a level's loads from memory inside the
    // march would be vector loads whose wait also drains the prefetch): dz,
    // 1/dz, the centre spacing above (0 at the top), the four reference steps
    // of T (see dtr) and with salinity those of S and the two linear
    // equation-of-state coefficients; the FP64 thickness for the FP64 sums.
    constexpr int LV_DZ = 0, LV_IDZ = 1, LV_DZC = 2, LV_T = 3, LV_S = 7, LV_ET = 11, LV_ES = 12;
    constexpr int NLV = SALT ? 13 : 7;
    constexpr bool kF32 = sizeof(R) == 4;
    __shared__ R sLev[kMaxLevels][NLV];
    __shared__ double sDzD[kF32 ? kMaxLevels : 1];

    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int i0 = bx * (TX - 1), j0 = by * (TY - 1);
    const int pi = i0 - 1 + tx, pj = j0 - 1 + ty;
    const int nx = S.nx, ny = S.ny, nz = S.nz, h = S.h;
    const bool used = (pi < nx) && (pj < ny);
    const bool cell = used && tx >= 1 && ty >= 1;
    const bool tcell = used && (tx >= 1 || ty >= 1);  // forms the tracer tendency of its column
    const bool need_x = used && ty >= 1;  // quantities a cell reads from its west neighbour
    const bool need_y = used && tx >= 1;  // ... from its south neighbour
    const bool need_c = need_x || need_y;

    const R* __restrict__ gT = f3<R>(S.t);
    const R* __restrict__ gU = f3<R>(S.u);
    const R* __restrict__ gV = f3<R>(S.v);
    const R* __restrict__ dtr = static_cast<const R*>(S.dtr);
    const R* __restrict__ gS = SALT ? f3<R>(S.s) : nullptr;
    const R* __restrict__ dsr = SALT ? static_cast<const R*>(S.dsr) : nullptr;
    const R* __restrict__ eost = SALT ? static_cast<const R*>(S.eos_tab) : nullptr;

    for (int q = tid; q < S.nz; q += NT) {
        sLev[q][LV_DZ] = R(S.dz[q]);
        sLev[q][LV_IDZ] = inv_level(S.dz[q], R(0));
        sLev[q][LV_DZC] = (q + 1 < S.nz) ? R(S.dzc[q + 1]) : R(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) sLev[q][LV_T + j] = dtr[q * 4 + j];
        if constexpr (SALT) {
#pragma unroll
            for (int j = 0; j < 4; ++j) sLev[q][LV_S + j] = dsr[q * 4 + j];
            sLev[q][LV_ET] = eost[2 * q];
            sLev[q][LV_ES] = eost[2 * q + 1];
        }
        if constexpr (kF32) sDzD[q] = S.dz[q];
    }
    auto dz_d = [&](int kk) -> double {
        if constexpr (kF32) return sDzD[kk];
        else return sLev[kk][LV_DZ];
    };
    // wet-layer counts of the tile (static over the march), origin (i0-4, j0-4)
    for (int q = tid; q < KN; q += NT) {
        const int li = q % KW, lj = q / KW;
        const int gi = min(max(i0 - 4 + li, -S.hk), nx + S.hk - 1);
        const int gj = min(max(j0 - 4 + lj, -S.hk), ny + S.hk - 1);
        sK[q] = S.kb[idxk(S, gi, gj)];
    }
    // this thread's slots of the value tiles (u, v origin (i0-3, j0-3); T origin
    // (i0-4, j0-4)), as offsets in a level
    int slot_off[NS], slot_offT[NST];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int e = tid + q * NT;
        const int li = e % LW, lj = e / LW;
        const int gi = min(max(i0 - 3 + li, -h), nx + h - 1);
        const int gj = min(max(j0 - 3 + lj, -h), ny + h - 1);
        slot_off[q] = gj * S.p3 + gi;
    }
#pragma unroll
    for (int q = 0; q < NST; ++q) {
        const int e = tid + q * NT;
        const int li = e % TW, lj = e / TW;
        // the point 4 cells before a periodic edge lies past a 3-cell halo:
        // read its interior image
        int gi = i0 - 4 + li, gj = j0 - 4 + lj;
        if (gi < -h) gi = S.periodic_x ? gi + nx : -h;
        if (gj < -h) gj = S.periodic_y ? gj + ny : -h;
        gi = min(gi, nx + h - 1);
        gj = min(gj, ny + h - 1);
        slot_offT[q] = gj * S.p3 + gi;
    }
    __syncthreads();

    const int me = (ty + 2) * LW + (tx + 2);   // this point in the u, v tiles
    const int meT = (ty + 3) * TW + (tx + 3);  // this point in the T tile
    const int mk = (ty + 3) * KW + (tx + 3);   // this point in the wet-count tile
    auto Kat = [&](int a, int b) { return sK[mk + a + b * KW]; };
    const int Kc = Kat(0, 0);
    const int Ku = min(Kc, Kat(-1, 0));
    const int Kv = min(Kc, Kat(0, -1));
    const int KuE = min(Kc, Kat(1, 0)), KuSE = min(Kat(0, -1), Kat(1, -1));
    const int KvN = min(Kc, Kat(0, 1)), KvNW = min(Kat(-1, 0), Kat(-1, 1));
    // smallest wet count over each horizontal stencil: all six points are
    // valid at level k when it reaches nz - k. The eight minima (each <= 128)
    // are kept as bytes of two registers.
    unsigned minA, minB;
    {
        int mTx = Kc, mTy = Kc, mux = Kc, muy = Kc, mvx = Kc, mvy = Kc, mTw = Kc, mTs = Kc;
#pragma unroll
        for (int r = -3; r <= 3; ++r) {
            mux = min(mux, Kat(r, 0));
            mvy = min(mvy, Kat(0, r));
            if (r >= -2) {
                mTx = min(mTx, Kat(r, 0));
                mTy = min(mTy, Kat(0, r));
                muy = min(muy, min(Kat(-1, r), Kat(0, r)));
                mvx = min(mvx, min(Kat(r, -1), Kat(r, 0)));
            }
            if (r <= 2) {  // the west and south faces of this point
                mTw = min(mTw, Kat(r, 0));
                mTs = min(mTs, Kat(0, r));
            }
        }
        minA = unsigned(mTx) | unsigned(mTy) << 8 | unsigned(mux) << 16 | unsigned(muy) << 24;
        minB = unsigned(mvx) | unsigned(mvy) << 8 | unsigned(mTw) << 16 | unsigned(mTs) << 24;
    }
    // vector-invariant form: smallest wet count over the cells around the six
    // corners of the u point's column (x -1..0, y -3..3) and of the v point's
    // row (x -3..3, y -1..0)
    unsigned minC = 0;
    if constexpr (VI) {
        int mzu = Kc, mzv = Kc;
#pragma unroll
        for (int r = -3; r <= 3; ++r) {
            mzu = min(mzu, min(Kat(-1, r), Kat(0, r)));
            mzv = min(mzv, min(Kat(r, -1), Kat(r, 0)));
        }
        minC = unsigned(mzu) | unsigned(mzv) << 8;
    }
    auto byte_of = [](unsigned v, int q) { return int((v >> (8 * q)) & 0xffu); };
#define mTx byte_of(minA, 0)
#define mTy byte_of(minA, 1)
#define mux byte_of(minA, 2)
#define muy byte_of(minA, 3)
#define mvx byte_of(minB, 0)
#define mvy byte_of(minB, 1)
#define mTw byte_of(minB, 2)
#define mTs byte_of(minB, 3)

    // row metrics of the point (clamped for points past the domain, which are unused)
    const int jr = min(max(pj, -h), ny + h - 2);
    const int ir = min(max(pi, -h), nx + h - 2);
    if (tx == 0) {
        sRow[0][ty] = R(S.dxv[jr]);
        sRow[1][ty] = R(S.dxv[jr + 1]);
        sRow[2][ty] = R(S.area[jr]);
        sRow[3][ty] = R(S.fcor[jr]);
        sRow[4][ty] = R(S.metric[jr]);
        sRow[5][ty] = R(1.0 / S.area[jr]);
        sRow[6][ty] = R(1.0 / (S.dxv[jr] * S.dy));
        sRow[7][ty] = R(1.0 / S.dxc[jr]);
        sRow[8][ty] = R(S.fcor_s[jr]);
    }
    if constexpr (VI) {
        if (tid < TY + 6) {
            const int row = min(max(j0 - 4 + tid, -h), ny + h - 1);
            sRX[0][tid] = R(S.dxc[row]);
            sRX[1][tid] = R(1.0 / (S.dxv[row] * S.dy * kZetaRef));
        }
    }
    const R dy = R(S.dy), inv_dy = R(1.0 / S.dy);
    const R ga = R(S.g * S.alpha);
    const R dt = R(S.dt);
    const R fbdt = R(S.pgf_w * S.dt);
    const R qT = R(S.eos_qT), qTS = R(S.eos_qTS), qS = R(S.eos_qS);
    const R c_new = first ? R(1) : R(1.5 + S.chi);
    const R c_old = first ? R(0) : R(0.5 + S.chi);

    // Surface value of the vertical transport: minus the divergence of the
    // depth-integrated transport of the current u, v (their column sums).
    double Wc = -(S.dy * (S.cu[idx2(S, ir + 1, jr)] - S.cu[idx2(S, ir, jr)]) +
                  S.dxv[jr + 1] * S.cv[idx2(S, ir, jr + 1)] - S.dxv[jr] * S.cv[idx2(S, ir, jr)]);
    sTop[tid] = R(Wc) * R(S.tref[nz - 1]);
    if constexpr (SALT) sTopS[tid] = R(Wc) * R(S.sref[nz - 1]);

    // own-column windows: w[r] holds level k + 2 - r
    R wt[6], wu[6], wv[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) { wt[r] = R(0); wu[r] = R(0); wv[r] = R(0); }
    const long long pl = S.plane3;
    // this column's offset in a level (a level's offset k * pl is uniform
    // across the workgroup); a ring column in a periodic halo is read at its
    // interior image, the only copy of its tracer history that is written
    const int hi = (pi < 0 && S.periodic_x) ? pi + nx : pi;
    const int hj = (pj < 0 && S.periodic_y) ? pj + ny : pj;
    int own = tcell ? hj * S.p3 + hi : 0;
    R ws[SALT ? 6 : 1];
#pragma unroll
    for (int r = 0; r < (SALT ? 6 : 1); ++r) ws[r] = R(0);
    if (tcell) {
#pragma unroll
        for (int r = 1; r < 6; ++r) {
            const int k = nz + 2 - r;  // before the first shift: levels nz+1 .. nz-3
            if (k >= 0 && k < nz) wt[r] = gT[k * pl + own];
            if constexpr (SALT)
                if (k >= 0 && k < nz) ws[r] = gS[k * pl + own];
        }
    }
    if (cell) {
#pragma unroll
        for (int r = 1; r < 6; ++r) {
            const int k = nz + 2 - r;
            if (k >= 0 && k < nz) { wu[r] = gU[k * pl + own]; wv[r] = gV[k * pl + own]; }
        }
    }
    // the level that enters the windows at the next shift (loaded a level ahead)
    R wtn = R(0), wun = R(0), wvn = R(0), wsn = R(0);
    if (nz - 4 >= 0) {
        const long long o = (long long)(nz - 4) * pl + own;
        if (tcell) wtn = gT[o];
        if constexpr (SALT)
            if (tcell) wsn = gS[o];
        if (cell) { wun = gU[o]; wvn = gV[o]; }
    }

    // prefetch of the top level's tile slots
    R pT[NST], pU[NS], pV[NS], pS[SALT ? NST : 1];
#pragma unroll
    for (int q = 0; q < NST; ++q) pT[q] = gT[(long long)(nz - 1) * pl + slot_offT[q]];
    if constexpr (SALT)
#pragma unroll
        for (int q = 0; q < NST; ++q) pS[q] = gS[(long long)(nz - 1) * pl + slot_offT[q]];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const long long o = (long long)(nz - 1) * pl + slot_off[q];
        pU[q] = gU[o]; pV[q] = gV[o];
    }

    R fzT_top = R(0), fzu_top = R(0), fzv_top = R(0);  // fluxes through the top face of level k
    R fzS_top = R(0);
    R Wm_top = R(0);                                     // masked W on that face
    R p_prev = R(0), b_prev = R(0);
    R GUp = R(0), GVp = R(0);  // momentum tendencies of level k+1 without the pressure gradient
    // vector-invariant form: the (f + zeta_hat) terms of the level, and the
    // vertical transports of the u and v control volumes on the top face
    R vi_u = R(0), vi_v = R(0), FuT = R(0), FvT = R(0);
    double gUacc = 0.0, gVacc = 0.0;
    const R rinv = R(S.restore_inv);
    R* __restrict__ gto = f3<R>(S.gt_out);
    const R* __restrict__ gti = f3<R>(S.gt);
    R* __restrict__ gup = f3<R>(S.gu);
    R* __restrict__ gvp = f3<R>(S.gv);
    R* __restrict__ tso = f3<R>(S.ts);
    R* __restrict__ uso = f3<R>(S.us);
    R* __restrict__ vso = f3<R>(S.vs);
    R* __restrict__ gso = SALT ? f3<R>(S.gs_out) : nullptr;
    const R* __restrict__ gsi = SALT ? f3<R>(S.gs) : nullptr;
    R* __restrict__ sso = SALT ? f3<R>(S.ss) : nullptr;

    // Completes the momentum step of level kk (one above the level being
    // marched) once the pressure of level kk of every point is in LDS:
    // AB2 of the other terms plus the forward-backward pressure gradient.
    // AB2 histories of the level being assembled (T, S) and of the level one
    // above (u, v: its momentum completes now), loaded with the next level's
    // tiles, before the level's barriers, so that no load in the march is
    // waited for right after it is issued (a wait drains every earlier load)
    R hgt = R(0), hgs = R(0), hgu = R(0), hgv = R(0);
    auto load_hist = [&](int k) {
        const long long o = (long long)k * pl + own;
        if (tcell) hgt = gti[o];
        if constexpr (SALT)
            if (tcell) hgs = gsi[o];
        if (cell && k + 1 < nz) { hgu = gup[o + pl]; hgv = gvp[o + pl]; }
    };
    auto finish_uv = [&](int kk, const R* P) {
        const int kw = nz - kk;
        const long long o = (long long)kk * pl + own;
        R hU = c_new * GUp - c_old * hgu;
        R hV = c_new * GVp - c_old * hgv;
        gup[o] = GUp;
        gvp[o] = GVp;
        if (Ku >= kw) hU -= (P[tid] - P[tid - 1]) * sRow[7][ty];
        if (Kv >= kw) hV -= (P[tid] - P[tid - TX]) * inv_dy;
        uso[o] = wu[1] + dt * hU;
        vso[o] = wv[1] + dt * hV;
        if (Ku >= kw) gUacc += dz_d(kk) * double(hU);
        if (Kv >= kw) gVacc += dz_d(kk) * double(hV);
    };

    for (int k = nz - 1; k >= 0; --k) {
        // The column and slot offsets are marked as redefined at every level so
        // that the compiler rebuilds each field's 64-bit address per level (two
        // instructions) instead of keeping a dozen of them live across the
        // march, which spilled registers.
        asm volatile("" : "+v"(own));
#pragma unroll
        for (int q = 0; q < NS; ++q) asm volatile("" : "+v"(slot_off[q]));
#pragma unroll
        for (int q = 0; q < NST; ++q) asm volatile("" : "+v"(slot_offT[q]));
        // shift the windows (level k-3 was loaded a level ahead)
#pragma unroll
        for (int r = 0; r < 5; ++r) { wt[r] = wt[r + 1]; wu[r] = wu[r + 1]; wv[r] = wv[r + 1]; }
        wt[5] = wtn; wu[5] = wun; wv[5] = wvn;
        if constexpr (SALT) {
#pragma unroll
            for (int r = 0; r < 5; ++r) ws[r] = ws[r + 1];
            ws[5] = wsn;
        }
        // stage level k from the prefetch registers, then issue every load
        // of the next level
        R* const sT = sT2[k & 1];
        R* const sU = sU2[k & 1];
        R* const sV = sV2[k & 1];
        R* const sS = sS2[SALT ? (k & 1) : 0];
#pragma unroll
        for (int q = 0; q < NST; ++q) {
            const int e = tid + q * NT;
            if (e < TN) sT[e] = pT[q];
            if constexpr (SALT)
                if (e < TN) sS[e] = pS[q];
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int e = tid + q * NT;
            if (e < LN) { sU[e] = pU[q]; sV[e] = pV[q]; }
        }
        load_hist(k);
        if (k >= 1) {
#pragma unroll
            for (int q = 0; q < NST; ++q) pT[q] = gT[(long long)(k - 1) * pl + slot_offT[q]];
            if constexpr (SALT)
#pragma unroll
                for (int q = 0; q < NST; ++q) pS[q] = gS[(long long)(k - 1) * pl + slot_offT[q]];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const long long o = (long long)(k - 1) * pl + slot_off[q];
                pU[q] = gU[o]; pV[q] = gV[o];
            }
        }
        wtn = R(0); wun = R(0); wvn = R(0); wsn = R(0);
        if (k - 4 >= 0) {
            const long long o = (long long)(k - 4) * pl + own;
            if (tcell) wtn = gT[o];
            if constexpr (SALT)
                if (tcell) wsn = gS[o];
            if (cell) { wun = gU[o]; wvn = gV[o]; }
        }
        __syncthreads();

        const R dzk = sLev[k][LV_DZ];
        const R inv_dz = sLev[k][LV_IDZ];
        const int kwet = nz - k;  // a column with K wet layers is wet at k iff K >= nz - k
        auto wet = [&](int a, int b) { return Kat(a, b) >= kwet; };
        auto mu = [&](int a, int b) { return wet(a, b) && wet(a - 1, b); };
        auto mv = [&](int a, int b) { return wet(a, b) && wet(a, b - 1); };
        auto at = [&](const R* f, int a, int b) { return f[me + a + b * LW]; };
        auto atT = [&](int a, int b) { return sT[meT + a + b * TW]; };

        // ---- quantities at this point ----
        if (used) {
            const R U00 = (Ku >= kwet) ? at(sU, 0, 0) * dy * dzk : R(0);
            const R U10 = (KuE >= kwet) ? at(sU, 1, 0) * dy * dzk : R(0);
            const R dxv1 = sRow[1][ty];
            const R V00 = (Kv >= kwet) ? at(sV, 0, 0) * sRow[0][ty] * dzk : R(0);
            const R V01 = (KvN >= kwet) ? at(sV, 0, 1) * dxv1 * dzk : R(0);
            R p[6];
            bool ok[6];
            // T through the east face (every point: the ring row's cells need it too)
            {
#pragma unroll
                for (int r = 0; r < 6; ++r) p[r] = atT(r - 2, 0);
                if (mTx >= kwet) fxT[tid] = (U10 == R(0)) ? R(0) : upwind_flux_wet(U10, p);
                else {
#pragma unroll
                    for (int r = 0; r < 6; ++r) ok[r] = wet(r - 2, 0);
                    fxT[tid] = upwind_flux(U10, p, ok);
                }
                if constexpr (SALT) {
#pragma unroll
                    for (int r = 0; r < 6; ++r) p[r] = sS[meT + r - 2];
                    if (mTx >= kwet) fxS[tid] = (U10 == R(0)) ? R(0) : upwind_flux_wet(U10, p);
                    else fxS[tid] = upwind_flux(U10, p, ok);
                }
            }
            // u through the cell centre (between u(pi) and u(pi+1)); in the
            // ring row: T through the south face (the vector-invariant form
            // only uses the ring row's)
            if (used && (VI ? (ty == 0 && tx >= 1) : (ty >= 1 || tx >= 1))) {
                const bool alt = ty == 0;
                const R* base = alt ? &sT[meT - 3 * TW] : &sU[me - 2];
                const int stride = alt ? TW : 1;
                const R F = alt ? V00 : R(0.5) * (U00 + U10);
#pragma unroll
                for (int r = 0; r < 6; ++r) p[r] = base[r * stride];
                if (alt ? (mTs >= kwet) : (mux >= kwet)) fxu[tid] = (F == R(0)) ? R(0) : upwind_flux_wet(F, p);
                else {
#pragma unroll
                    for (int r = 0; r < 6; ++r) ok[r] = alt ? wet(0, r - 3) : mu(r - 2, 0);
                    fxu[tid] = upwind_flux(F, p, ok);
                }
            }
            if (!VI && need_x) {
                const R U1m = (KuSE >= kwet) ? at(sU, 1, -1) * dy * dzk : R(0);
                // v through the south-east corner (between v(pi,pj) and v(pi+1,pj))
                const R Fv = R(0.5) * (U1m + U10);
#pragma unroll
                for (int r = 0; r < 6; ++r) p[r] = at(sV, r - 2, 0);
                if (mvx >= kwet) fxv[tid] = (Fv == R(0)) ? R(0) : upwind_flux_wet(Fv, p);
                else {
#pragma unroll
                    for (int r = 0; r < 6; ++r) ok[r] = mv(r - 2, 0);
                    fxv[tid] = upwind_flux(Fv, p, ok);
                }
            } else if constexpr (SALT) {
                if (used && ty == 0 && tx >= 1) {  // ring row: S through the south face
#pragma unroll
                    for (int r = 0; r < 6; ++r) p[r] = sS[meT + (r - 3) * TW];
                    if (mTs >= kwet) fxv[tid] = (V00 == R(0)) ? R(0) : upwind_flux_wet(V00, p);
                    else {
#pragma unroll
                        for (int r = 0; r < 6; ++r) ok[r] = wet(0, r - 3);
                        fxv[tid] = upwind_flux(V00, p, ok);
                    }
                }
            }
            // T through the north face (every point: the ring column's cells need it too)
            {
#pragma unroll
                for (int r = 0; r < 6; ++r) p[r] = atT(0, r - 2);
                if (mTy >= kwet) fyT[tid] = (V01 == R(0)) ? R(0) : upwind_flux_wet(V01, p);
                else {
#pragma unroll
                    for (int r = 0; r < 6; ++r) ok[r] = wet(0, r - 2);
                    fyT[tid] = upwind_flux(V01, p, ok);
                }
                if constexpr (SALT) {
#pragma unroll
                    for (int r = 0; r < 6; ++r) p[r] = sS[meT + (r - 2) * TW];
                    if (mTy >= kwet) fyS[tid] = (V01 == R(0)) ? R(0) : upwind_flux_wet(V01, p);
                    else fyS[tid] = upwind_flux(V01, p, ok);
                }
            }
            // u through the north-west corner (between u(pi,pj) and u(pi,pj+1));
            // in the ring column: T through the west face
            if (!VI || (tx == 0 && ty >= 1)) {
                const bool alt = tx == 0;
                const R Vm1 = (KvNW >= kwet) ? at(sV, -1, 1) * dxv1 * dzk : R(0);
                const R* base = alt ? &sT[meT - 3] : &sU[me - 2 * LW];
                const int stride = alt ? 1 : LW;
                const R F = alt ? U00 : R(0.5) * (Vm1 + V01);
#pragma unroll
                for (int r = 0; r < 6; ++r) p[r] = base[r * stride];
                if (alt ? (mTw >= kwet) : (muy >= kwet)) fyu[tid] = (F == R(0)) ? R(0) : upwind_flux_wet(F, p);
                else {
#pragma unroll
                    for (int r = 0; r < 6; ++r) ok[r] = alt ? wet(r - 3, 0) : mu(0, r - 2);
                    fyu[tid] = upwind_flux(F, p, ok);
                }
            }
            if (!VI && need_y) {
                // v through the cell centre (between v(pj) and v(pj+1))
                const R Fv = R(0.5) * (V00 + V01);
#pragma unroll
                for (int r = 0; r < 6; ++r) p[r] = at(sV, 0, r - 2);
                if (mvy >= kwet) fyv[tid] = (Fv == R(0)) ? R(0) : upwind_flux_wet(Fv, p);
                else {
#pragma unroll
                    for (int r = 0; r < 6; ++r) ok[r] = mv(0, r - 2);
                    fyv[tid] = upwind_flux(Fv, p, ok);
                }
            } else if constexpr (SALT) {
                if (used && tx == 0 && ty >= 1) {  // ring column: S through the west face
#pragma unroll
                    for (int r = 0; r < 6; ++r) p[r] = sS[meT + r - 3];
                    if (mTw >= kwet) fyv[tid] = (U00 == R(0)) ? R(0) : upwind_flux_wet(U00, p);
                    else {
#pragma unroll
                        for (int r = 0; r < 6; ++r) ok[r] = wet(r - 3, 0);
                        fyv[tid] = upwind_flux(U00, p, ok);
                    }
                }
            }
            if (!VI && need_c) {
                // Coriolis: Q = (f + u_c tan(phi)/a) V_c on wet cells
                const R uc = R(0.5) * (at(sU, 0, 0) + at(sU, 1, 0));
                const R vc = R(0.5) * (at(sV, 0, 0) + at(sV, 0, 1));
                const R Q = (Kc >= kwet) ? (sRow[3][ty] + sRow[4][ty] * uc) * sRow[2][ty] * dzk : R(0);
                sQv[tid] = Q * vc;
                sQu[tid] = Q * uc;
            }
            if constexpr (VI) {
                auto muu = [&](int a, int b) { return mu(a, b) ? at(sU, a, b) : R(0); };
                auto mvv = [&](int a, int b) { return mv(a, b) ? at(sV, a, b) : R(0); };
                {  // kinetic energy at this point
                    const R uw = muu(0, 0), ue = muu(1, 0), vs = mvv(0, 0), vn = mvv(0, 1);
                    sKE[tid] = R(0.25) * (uw * uw + ue * ue) + R(0.25) * (vs * vs + vn * vn);
                }
                if (cell) {
                    // corner (pi+a, pj+b), the south-west corner of cell (pi+a, pj+b):
                    // its circulation over dxv dy zeta_ref, 0 where it touches land
                    auto cwet = [&](int a, int b) {
                        return wet(a - 1, b - 1) && wet(a, b - 1) && wet(a - 1, b) && wet(a, b);
                    };
                    auto zc = [&](int a, int b) {
                        const int rr = ty + 3 + b;
                        const R circ = dy * (at(sV, a, b) - at(sV, a - 1, b)) -
                                       (sRX[0][rr] * at(sU, a, b) - sRX[0][rr - 1] * at(sU, a, b - 1));
                        return circ * sRX[1][rr];
                    };
                    const R vbar = R(0.25) * (mvv(-1, 0) + mvv(-1, 1) + mvv(0, 0) + mvv(0, 1));
                    const R ubar = R(0.25) * (muu(0, -1) + muu(1, -1) + muu(0, 0) + muu(1, 0));
                    R zu, zv;
                    if (int(minC & 0xffu) >= kwet) {  // the six corners along y
#pragma unroll
                        for (int r = 0; r < 6; ++r) p[r] = zc(0, r - 2);
                        zu = upwind_value_wet(vbar, p);
                    } else {
#pragma unroll
                        for (int r = 0; r < 6; ++r) {
                            ok[r] = cwet(0, r - 2);
                            p[r] = ok[r] ? zc(0, r - 2) : R(0);
                        }
                        zu = upwind_value(vbar, p, ok);
                    }
                    if (int((minC >> 8) & 0xffu) >= kwet) {  // the six corners along x
#pragma unroll
                        for (int r = 0; r < 6; ++r) p[r] = zc(r - 2, 0);
                        zv = upwind_value_wet(ubar, p);
                    } else {
#pragma unroll
                        for (int r = 0; r < 6; ++r) {
                            ok[r] = cwet(r - 2, 0);
                            p[r] = ok[r] ? zc(r - 2, 0) : R(0);
                        }
                        zv = upwind_value(ubar, p, ok);
                    }
                    vi_u = (sRow[3][ty] + R(kZetaRef) * zu) * vbar;
                    vi_v = -(sRow[8][ty] + R(kZetaRef) * zv) * ubar;
                }
            }
            // vertical transport on the bottom face of level k
            const double div = double(U10) - double(U00) + (double(V01) - double(V00));
            Wc = Wc + div;
            const bool mw = (k >= 1) && (Kc >= kwet + 1);  // layers k-1 and k both wet
            sWm[tid] = mw ? R(Wc) : R(0);
        }
        __syncthreads();

        // ---- assembly: tracer of every column with a tendency, momentum of the cells ----
        const R Wm_b = sWm[tid];
        R* const Pk = &sP[(k & 1) * NT];
        if (tcell) {
            const int c = tid, cw = tid - 1, cs = tid - TX;

            // vertical fluxes through the bottom face (between levels k-1 and k)
            R fzT_bot = R(0), fzu_bot = R(0), fzv_bot = R(0);
            R E_bot = R(0), fzS_bot = R(0), ES_bot = R(0);
            R Fu_b = R(0), Fv_b = R(0);  // vertical transports of the u, v control volumes
            if (k >= 1) {
                // levels k-3 .. k+2 all inside the column: the open-ocean path
                const bool zin = (k >= 3) && (k + 2 < nz);
                if (Wm_b != R(0)) {
                    // reconstruct the full tracer from differences relative to the
                    // upwind cell (anomaly steps plus reference-profile steps)
                    const bool pos = Wm_b > R(0);
                    const int kc = pos ? k - 1 : k;
                    const int la = pos ? k - 3 : k + 2, lb = pos ? k - 2 : k + 1;
                    const int ld = pos ? k : k - 1, le = pos ? k + 1 : k - 2;
                    auto okl = [&](int l) { return l >= 0 && l < nz && Kc >= nz - l; };
                    const bool open = zin && Kc >= nz - (k - 3);
                    auto zflux = [&](const R* w, const int tab, R& Eb) {
                        const R ta = pos ? w[5] : w[0], tb = pos ? w[4] : w[1], tcv = pos ? w[3] : w[2];
                        const R td = pos ? w[2] : w[3], te = pos ? w[1] : w[4];
                        const R* st = &sLev[kc][tab];
                        const R da = (ta - tcv) + (pos ? st[0] : st[3]);
                        const R db = (tb - tcv) + (pos ? st[1] : st[2]);
                        const R dd = (td - tcv) + (pos ? st[2] : st[1]);
                        const R de = (te - tcv) + (pos ? st[3] : st[0]);
                        const R rel = open ? weno5z(da, db, R(0), dd, de)
                                           : recon(da, db, R(0), dd, de, okl(la), okl(lb), true, okl(ld), okl(le));
                        // reference profile carried through this face, relative to the level's reference
                        Eb = pos ? Wm_b * (-sLev[k][tab + 1]) : R(0);
                        return Wm_b * (tcv + rel);
                    };
                    fzT_bot = zflux(wt, LV_T, E_bot);
                    if constexpr (SALT) fzS_bot = zflux(ws, LV_S, ES_bot);
                }
                if (cell) {
                    const R Fu = R(0.5) * (sWm[cw] + Wm_b);
                    Fu_b = Fu;
                    if (Fu != R(0)) {
                        R pu[6];
#pragma unroll
                        for (int r = 0; r < 6; ++r) pu[r] = wu[5 - r];
                        if (zin && Ku >= nz - (k - 3)) {
                            fzu_bot = upwind_flux_wet(Fu, pu);
                        } else {
                            bool oku[6];
#pragma unroll
                            for (int r = 0; r < 6; ++r) {
                                const int l = k - 3 + r;
                                oku[r] = (l >= 0 && l < nz && Ku >= nz - l);
                            }
                            fzu_bot = upwind_flux(Fu, pu, oku);
                        }
                    }
                    const R Fv = R(0.5) * (sWm[cs] + Wm_b);
                    Fv_b = Fv;
                    if (Fv != R(0)) {
                        R pv[6];
#pragma unroll
                        for (int r = 0; r < 6; ++r) pv[r] = wv[5 - r];
                        if (zin && Kv >= nz - (k - 3)) {
                            fzv_bot = upwind_flux_wet(Fv, pv);
                        } else {
                            bool okv[6];
#pragma unroll
                            for (int r = 0; r < 6; ++r) {
                                const int l = k - 3 + r;
                                okv[r] = (l >= 0 && l < nz && Kv >= nz - l);
                            }
                            fzv_bot = upwind_flux(Fv, pv, okv);
                        }
                    }
                }
            }

            // tracer; a ring column takes its far-face flux from its own idle slot
            R GT = R(0);
            if (Kc >= kwet) {
                R E_top;
                if (k == nz - 1) {
                    E_top = sTop[c];
                } else {
                    // upwind cell k+1 when the face transport is downward
                    E_top = (Wm_top > R(0)) ? R(0) : Wm_top * (-sLev[k][LV_T + 2]);
                }
                const R fw = (tx == 0) ? fyu[c] : fxT[cw];
                const R fs = (ty == 0) ? fxu[c] : fyT[cs];
                const R divF = (fxT[c] - fw) + (fyT[c] - fs) + (fzT_top - fzT_bot);
                GT = (-divF + (E_top - E_bot)) * (sRow[5][ty] * inv_dz);
                if (k == nz - 1) GT += (R(S.tstar[idx2(S, pi, pj)]) - wt[2]) * rinv;
            }
            // salinity the same way; the ring's far-face fluxes sit in the v slots
            R GS = R(0);
            if constexpr (SALT) {
                if (Kc >= kwet) {
                    R ES_top;
                    if (k == nz - 1) ES_top = sTopS[c];
                    else ES_top = (Wm_top > R(0)) ? R(0) : Wm_top * (-sLev[k][LV_S + 2]);
                    const R fw = (tx == 0) ? fyv[c] : fxS[cw];
                    const R fs = (ty == 0) ? fxv[c] : fyS[cs];
                    const R divF = (fxS[c] - fw) + (fyS[c] - fs) + (fzS_top - fzS_bot);
                    GS = (-divF + (ES_top - ES_bot)) * (sRow[5][ty] * inv_dz);
                    if (k == nz - 1) GS += (R(S.sstar[idx2(S, pi, pj)]) - ws[2]) * rinv;
                }
            }
            // AB2 of the tracer (G^n goes to the other history buffer), and the
            // pressure of T^n + eps dt Ghat_T from p = 0 at z = 0 downward
            const R hT = c_new * GT - c_old * hgt;
            const long long o = (long long)k * pl + own;
            if (cell) {
                gto[o] = GT;
                tso[o] = wt[2] + dt * hT;
            }
            R b;
            if constexpr (SALT) {
                // buoyancy anomaly of T' + eps dt Ghat_T, S' + eps dt Ghat_S
                // (quadratic equation of state about the level's reference water)
                const R hS = c_new * GS - c_old * hgs;
                if (cell) {
                    gso[o] = GS;
                    sso[o] = ws[2] + dt * hS;
                }
                const R tf = wt[2] + fbdt * hT, sf = ws[2] + fbdt * hS;
                b = tf * (sLev[k][LV_ET] + qT * tf + qTS * sf) + sf * (sLev[k][LV_ES] + qS * sf);
            } else {
                b = ga * (wt[2] + fbdt * hT);
            }
            const R pk = (k == nz - 1) ? -R(0.5) * dzk * b : p_prev - sLev[k][LV_DZC] * (R(0.5) * (b + b_prev));
            p_prev = pk;
            b_prev = b;
            Pk[tid] = pk;

            // momentum of the cells: level k+1 completes with its pressure
            // (written one level earlier); level k waits for its own
            if (cell) {
                if (k + 1 < nz) finish_uv(k + 1, &sP[((k + 1) & 1) * NT]);
                R GUm = R(0);
                if (Ku >= kwet) {
                    const R ivol = sRow[5][ty] * inv_dz;
                    if constexpr (VI) {
                        // (f + zeta_hat) vbar - dK/dx - w du/dz
                        GUm = vi_u - (sKE[c] - sKE[cw]) * sRow[7][ty] -
                              ((fzu_top - fzu_bot) - wu[2] * (FuT - Fu_b)) * ivol;
                    } else {
                        const R divF = (fxu[c] - fxu[cw]) + (fyu[c] - fyu[cs]) + (fzu_top - fzu_bot);
                        GUm = -divF * ivol + (sQv[cw] + sQv[c]) * (R(0.5) * ivol);
                    }
                    if (k == nz - 1) GUm += R(S.taux[idx2(S, pi, pj)] / (S.rho0 * S.dz[nz - 1]));
                }
                R GVm = R(0);
                if (Kv >= kwet) {
                    const R ivol = sRow[6][ty] * inv_dz;
                    if constexpr (VI) {
                        // -(f + zeta_hat) ubar - dK/dy - w dv/dz
                        GVm = vi_v - (sKE[c] - sKE[cs]) * inv_dy -
                              ((fzv_top - fzv_bot) - wv[2] * (FvT - Fv_b)) * ivol;
                    } else {
                        const R divF = (fxv[c] - fxv[cw]) + (fyv[c] - fyv[cs]) + (fzv_top - fzv_bot);
                        GVm = -divF * ivol - (sQu[cs] + sQu[c]) * (R(0.5) * ivol);
                    }
                    if (k == nz - 1) GVm += R(S.tauy[idx2(S, pi, pj)] / (S.rho0 * S.dz[nz - 1]));
                }
                GUp = GUm;
                GVp = GVm;
            }

            fzT_top = fzT_bot;
            if constexpr (SALT) fzS_top = fzS_bot;
            fzu_top = fzu_bot;
            fzv_top = fzv_bot;
            if constexpr (VI) {
                FuT = Fu_b;
                FvT = Fv_b;
            }
        }
        Wm_top = Wm_b;
    }
    __syncthreads();
    // the bottom level's pressure is in LDS after this barrier; the window
    // is shifted once more so that w[1] holds level 0
    if (cell) {
        hgu = gup[own];  // level 0
        hgv = gvp[own];
#pragma unroll
        for (int r = 0; r < 5; ++r) { wu[r] = wu[r + 1]; wv[r] = wv[r + 1]; }
        finish_uv(0, &sP[0]);
        S.gU[idx2(S, pi, pj)] = gUacc;
        S.gV[idx2(S, pi, pj)] = gVacc;
    }
#undef mTx
#undef mTy
#undef mux
#undef muy
#undef mvx
#undef mvy
#undef mTw
#undef mTs
}

template <typename R, int TX, int TY, bool SALT, bool VI>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(TendWaves<R, SALT || VI, TY>::n)))
void k_tend(const DevState S, const int first, const int gx) {
    const int2 t = band_tile(xcd_tile(blockIdx.x, gridDim.x), gx, gridDim.x / gx);
    tend_tile<R, TX, TY, SALT, VI>(S, first, t.x, t.y);
}

// Ensemble: entry b of the tile table names (member, bx, by); the host orders
// the table so that each XCD receives contiguous tiles of a member.
template <typename R, int TY>
__global__ __launch_bounds__(TXB * TY) __attribute__((amdgpu_waves_per_eu(TendWaves<R, false, TY>::n)))
void k_tend_batched(const DevState* __restrict__ members, const int4* __restrict__ tiles, const int first) {
    const int4 e = tiles[blockIdx.x];
    tend_tile<R, TXB, TY, false, false>(members[e.x], first, e.y, e.z);
}

// The same over a queue of table entries, with persistent workgroups.
template <typename R, int TY>
__global__ __launch_bounds__(TXB * TY) __attribute__((amdgpu_waves_per_eu(TendWaves<R, false, TY>::n)))
void k_tend_queued(const DevState* __restrict__ members, const int4* __restrict__ tiles, const int ntiles,
                   const int first, int* __restrict__ queue) {
    for_each_queued_tile(queue, ntiles, [&](int b) {
        const int4 e = tiles[b];
        tend_tile<R, TXB, TY, false, false>(members[e.x], first, e.y, e.z);
    });
}

// Rows of the 64-wide ensemble tiles: 4 or 8 as chosen, else 8 in FP32 and 4 in FP64.
int tend_tile_rows(int precision_bytes, int ty_choice) {
    if (ty_choice == 4 || ty_choice == 8) return ty_choice;
    return precision_bytes == 4 ? 8 : 4;
}

template <typename R, int TX, int TY, bool SALT, bool VI>
hipError_t launch_tend_shape(const DevState& s, int first, hipStream_t st) {
    const int gx = (s.nx + TX - 2) / (TX - 1);
    const int gy = (s.ny + TY - 2) / (TY - 1);
    hipLaunchKernelGGL((k_tend<R, TX, TY, SALT, VI>), dim3(gx * gy), dim3(TX, TY), 0, st, s, first, gx);
    return hipGetLastError();
}

// Single state: the precision's shape; with salinity or the vector-invariant
// form the wider-register shape; a 64-wide tile of 4 or 8 rows when chosen
// (temperature only, flux form).
template <typename R>
hipError_t launch_tendency(const DevState& s, int first, hipStream_t st) {
    constexpr int WX = TendShapeSalt<R>::TX, WY = TendShapeSalt<R>::TY;
    if (s.salinity && s.vi) return launch_tend_shape<R, WX, WY, true, true>(s, first, st);
    if (s.salinity) return launch_tend_shape<R, WX, WY, true, false>(s, first, st);
    if (s.vi) return launch_tend_shape<R, TendShape<R>::TX, TendShape<R>::TY, false, true>(s, first, st);
    if (s.tend_ty == 8) return launch_tend_shape<R, TXB, 8, false, false>(s, first, st);
    if (s.tend_ty == 4) return launch_tend_shape<R, TXB, 4, false, false>(s, first, st);
    return launch_tend_shape<R, TendShape<R>::TX, TendShape<R>::TY, false, false>(s, first, st);
}

template <typename R>
hipError_t launch_tendency_batched(const DevState* members, const int4* tiles, int ntiles, int ty, int first,
                                   int* queue, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (queue) {
        if (ty == 8) {
            const int nb = std::min(ntiles, resident_workgroups((const void*)k_tend_queued<R, 8>, TXB * 8));
            hipLaunchKernelGGL((k_tend_queued<R, 8>), dim3(nb), dim3(TXB, 8), 0, st, members, tiles, ntiles, first,
                               queue);
        } else {
            const int nb = std::min(ntiles, resident_workgroups((const void*)k_tend_queued<R, 4>, TXB * 4));
            hipLaunchKernelGGL((k_tend_queued<R, 4>), dim3(nb), dim3(TXB, 4), 0, st, members, tiles, ntiles, first,
                               queue);
        }
        return hipGetLastError();
    }
    if (ty == 8) hipLaunchKernelGGL((k_tend_batched<R, 8>), dim3(ntiles), dim3(TXB, 8), 0, st, members, tiles, first);
    else hipLaunchKernelGGL((k_tend_batched<R, 4>), dim3(ntiles), dim3(TXB, 4), 0, st, members, tiles, first);
    return hipGetLastError();
}

template hipError_t launch_tendency<double>(const DevState&, int, hipStream_t);
template hipError_t launch_tendency<float>(const DevState&, int, hipStream_t);
template hipError_t launch_tendency_batched<double>(const DevState*, const int4*, int, int, int, int*, hipStream_t);
template hipError_t launch_tendency_batched<float>(const DevState*, const int4*, int, int, int, int*, hipStream_t);

}  // namespace ocn
