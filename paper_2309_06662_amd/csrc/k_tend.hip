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
// Mapping. A 64x4 workgroup owns a tile of (64-1) x (4-1) columns and marches
// from the surface to the bottom. Thread (tx, ty) sits on point
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

namespace ocn {

constexpr int TX = 64;
constexpr int TY = 4;
constexpr int LW = TX + 5;   // tile columns: points i0-1-2 .. i0-1+TX-1+3
constexpr int LH = TY + 5;
constexpr int LN = LW * LH;
constexpr int KW = TX + 6;   // wet-count tile: one more column and row on the low side,
constexpr int KH = TY + 6;   // for the masks of velocity points at the stencil ends
constexpr int KN = KW * KH;

template <typename R> struct Eps;
template <> struct Eps<double> { static constexpr double v = 1e-8; };
template <> struct Eps<float> { static constexpr float v = 1e-8f; };

// Fifth-order WENO-Z face value (Borges et al. 2008) on Jiang-Shu smoothness
// indicators; c is the upwind cell, the face lies between c and d.
template <typename R>
__device__ __forceinline__ R weno5z(R a, R b, R c, R d, R e) {
    const R sixth = R(1) / R(6);
    const R q0 = (R(2) * a - R(7) * b + R(11) * c) * sixth;
    const R q1 = (-b + R(5) * c + R(2) * d) * sixth;
    const R q2 = (R(2) * c + R(5) * d - e) * sixth;
    const R s0 = a - R(2) * b + c, r0 = a - R(4) * b + R(3) * c;
    const R s1 = b - R(2) * c + d, r1 = b - d;
    const R s2 = c - R(2) * d + e, r2 = R(3) * c - R(4) * d + e;
    const R k13 = R(13) / R(12);
    const R b0 = k13 * s0 * s0 + R(0.25) * r0 * r0;
    const R b1 = k13 * s1 * s1 + R(0.25) * r1 * r1;
    const R b2 = k13 * s2 * s2 + R(0.25) * r2 * r2;
    const R tau = fabs(b0 - b2);
    const R z0 = tau / (b0 + Eps<R>::v);
    const R z1 = tau / (b1 + Eps<R>::v);
    const R z2 = tau / (b2 + Eps<R>::v);
    const R a0 = R(0.1) * (R(1) + z0 * z0);
    const R a1 = R(0.6) * (R(1) + z1 * z1);
    const R a2 = R(0.3) * (R(1) + z2 * z2);
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// Third-order WENO-JS face value on (b, c, d), c upwind.
template <typename R>
__device__ __forceinline__ R weno3(R b, R c, R d) {
    const R q0 = R(0.5) * (R(3) * c - b);
    const R q1 = R(0.5) * (c + d);
    const R e0 = (c - b) * (c - b) + Eps<R>::v;
    const R e1 = (d - c) * (d - c) + Eps<R>::v;
    const R a0 = (R(1) / R(3)) / (e0 * e0);
    const R a1 = (R(2) / R(3)) / (e1 * e1);
    return (a0 * q0 + a1 * q1) / (a0 + a1);
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
// around it (face between points -1 and 0).
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

template <typename R>
__global__ __launch_bounds__(TX * TY) void k_tend(const DevState S, const int first) {
    __shared__ R sT[LN], sU[LN], sV[LN];
    __shared__ int sK[KN];
    __shared__ R fxT[TY * TX], fyT[TY * TX], fxu[TY * TX], fyu[TY * TX], fxv[TY * TX], fyv[TY * TX];
    __shared__ R sQv[TY * TX], sQu[TY * TX], sP[TY * TX], sWm[TY * TX];

    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int i0 = blockIdx.x * (TX - 1), j0 = blockIdx.y * (TY - 1);
    const int pi = i0 - 1 + tx, pj = j0 - 1 + ty;
    const int nx = S.nx, ny = S.ny, nz = S.nz, h = S.h;
    const bool used = (pi < nx) && (pj < ny);
    const bool cell = used && tx >= 1 && ty >= 1;

    const R* __restrict__ gT = f3<R>(S.t);
    const R* __restrict__ gU = f3<R>(S.u);
    const R* __restrict__ gV = f3<R>(S.v);
    const R* __restrict__ dtr = static_cast<const R*>(S.dtr);

    // wet-layer counts of the tile (static over the march), origin (i0-4, j0-4)
    for (int q = tid; q < KN; q += TX * TY) {
        const int li = q % KW, lj = q / KW;
        const int gi = min(max(i0 - 4 + li, -h), nx + h - 1);
        const int gj = min(max(j0 - 4 + lj, -h), ny + h - 1);
        sK[q] = S.kb[idxk(S, gi, gj)];
    }
    __syncthreads();

    const int me = (ty + 2) * LW + (tx + 2);   // this point in the value tiles
    const int mk = (ty + 3) * KW + (tx + 3);   // this point in the wet-count tile
    const int Kc = sK[mk];
    const int Ku = min(Kc, sK[mk - 1]);
    const int Kv = min(Kc, sK[mk - KW]);

    // row metrics of the point (clamped for points past the domain, which are unused)
    const int jr = min(max(pj, -h), ny + h - 2);
    const int ir = min(max(pi, -h), nx + h - 2);
    const R dxc = R(S.dxc[jr]), dxv0 = R(S.dxv[jr]), dxv1 = R(S.dxv[jr + 1]);
    const R area = R(S.area[jr]), fc = R(S.fcor[jr]), met = R(S.metric[jr]);
    const R dy = R(S.dy);
    const R ga = R(S.g * S.alpha);
    const R dt = R(S.dt);
    const R c_new = first ? R(1) : R(1.5 + S.chi);
    const R c_old = first ? R(0) : R(0.5 + S.chi);

    // Surface value of the vertical transport: minus the divergence of the
    // depth-integrated transport of the current u, v (their column sums).
    double Wc = -(S.dy * (S.cu[idx2(S, ir + 1, jr)] - S.cu[idx2(S, ir, jr)]) +
                  S.dxv[jr + 1] * S.cv[idx2(S, ir, jr + 1)] - S.dxv[jr] * S.cv[idx2(S, ir, jr)]);
    const double Wsurf = Wc;

    // own-column windows: w[r] holds level k + 2 - r
    R wt[6], wu[6], wv[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) { wt[r] = R(0); wu[r] = R(0); wv[r] = R(0); }
    if (cell) {
#pragma unroll
        for (int r = 1; r < 6; ++r) {
            const int k = nz + 2 - r;  // before the first shift: levels nz+1 .. nz-3
            if (k >= 0 && k < nz) {
                const long long o = idx3(S, pi, pj, k);
                wt[r] = gT[o]; wu[r] = gU[o]; wv[r] = gV[o];
            }
        }
    }

    R fzT_top = R(0), fzu_top = R(0), fzv_top = R(0);  // fluxes through the top face of level k
    R Wm_top = R(0);                                     // masked W on that face
    R p_prev = R(0), b_prev = R(0);
    double gUacc = 0.0, gVacc = 0.0;
    const long long pl = S.plane3;
    const R wind_u = cell ? R(S.taux[idx2(S, pi, pj)] / (S.rho0 * S.dz[nz - 1])) : R(0);
    const R wind_v = cell ? R(S.tauy[idx2(S, pi, pj)] / (S.rho0 * S.dz[nz - 1])) : R(0);
    const R tstar = cell ? R(S.tstar[idx2(S, pi, pj)]) : R(0);
    const R rinv = R(S.restore_inv);

    for (int k = nz - 1; k >= 0; --k) {
        // shift the windows and load level k-3
#pragma unroll
        for (int r = 0; r < 5; ++r) { wt[r] = wt[r + 1]; wu[r] = wu[r + 1]; wv[r] = wv[r + 1]; }
        wt[5] = R(0); wu[5] = R(0); wv[5] = R(0);
        if (cell && k - 3 >= 0) {
            const long long o = idx3(S, pi, pj, k - 3);
            wt[5] = gT[o]; wu[5] = gU[o]; wv[5] = gV[o];
        }
        // stage level k of the tile
        for (int q = tid; q < LN; q += TX * TY) {
            const int li = q % LW, lj = q / LW;
            const int gi = min(max(i0 - 3 + li, -h), nx + h - 1);
            const int gj = min(max(j0 - 3 + lj, -h), ny + h - 1);
            const long long o = (long long)k * pl + (long long)gj * S.p3 + gi;
            sT[q] = gT[o]; sU[q] = gU[o]; sV[q] = gV[o];
        }
        __syncthreads();

        const R dzk = R(S.dz[k]);
        const int kwet = nz - k;  // a column with K wet layers is wet at k iff K >= nz - k
        // masks at offset (a, b) from this point
        auto wet = [&](int a, int b) { return sK[mk + a + b * KW] >= kwet; };
        auto mu = [&](int a, int b) { return wet(a, b) && wet(a - 1, b); };
        auto mv = [&](int a, int b) { return wet(a, b) && wet(a, b - 1); };
        auto U3 = [&](int a, int b) { return mu(a, b) ? sU[me + a + b * LW] * dy * dzk : R(0); };
        auto V3 = [&](int a, int b, R dxv) { return mv(a, b) ? sV[me + a + b * LW] * dxv * dzk : R(0); };

        // ---- quantities at this point ----
        {
            const R U00 = U3(0, 0), U10 = U3(1, 0), U1m = U3(1, -1);
            const R V00 = V3(0, 0, dxv0), V01 = V3(0, 1, dxv1), Vm1 = V3(-1, 1, dxv1);
            R p[6];
            bool ok[6];
            // T through the east face
#pragma unroll
            for (int r = 0; r < 6; ++r) { p[r] = sT[me - 2 + r]; ok[r] = wet(r - 2, 0); }
            fxT[tid] = upwind_flux(U10, p, ok);
            // T through the north face
#pragma unroll
            for (int r = 0; r < 6; ++r) { p[r] = sT[me + (r - 2) * LW]; ok[r] = wet(0, r - 2); }
            fyT[tid] = upwind_flux(V01, p, ok);
            // u through the cell centre (between u(pi) and u(pi+1))
#pragma unroll
            for (int r = 0; r < 6; ++r) { p[r] = sU[me - 2 + r]; ok[r] = mu(r - 2, 0); }
            fxu[tid] = upwind_flux(R(0.5) * (U00 + U10), p, ok);
            // u through the north-west corner (between u(pi,pj) and u(pi,pj+1))
#pragma unroll
            for (int r = 0; r < 6; ++r) { p[r] = sU[me + (r - 2) * LW]; ok[r] = mu(0, r - 2); }
            fyu[tid] = upwind_flux(R(0.5) * (Vm1 + V01), p, ok);
            // v through the south-east corner (between v(pi,pj) and v(pi+1,pj))
#pragma unroll
            for (int r = 0; r < 6; ++r) { p[r] = sV[me - 2 + r]; ok[r] = mv(r - 2, 0); }
            fxv[tid] = upwind_flux(R(0.5) * (U1m + U10), p, ok);
            // v through the cell centre (between v(pj) and v(pj+1))
#pragma unroll
            for (int r = 0; r < 6; ++r) { p[r] = sV[me + (r - 2) * LW]; ok[r] = mv(0, r - 2); }
            fyv[tid] = upwind_flux(R(0.5) * (V00 + V01), p, ok);

            // Coriolis: Q = (f + u_c tan(phi)/a) V_c on wet cells
            const R uc = R(0.5) * (sU[me] + sU[me + 1]);
            const R vc = R(0.5) * (sV[me] + sV[me + LW]);
            const R Q = wet(0, 0) ? (fc + met * uc) * area * dzk : R(0);
            sQv[tid] = Q * vc;
            sQu[tid] = Q * uc;

            // hydrostatic pressure of the anomaly, from p = 0 at z = 0 downward
            const R b = ga * sT[me];
            const R pk = (k == nz - 1) ? -R(0.5) * dzk * b : p_prev - R(S.dzc[k + 1]) * (R(0.5) * (b + b_prev));
            p_prev = pk;
            b_prev = b;
            sP[tid] = pk;

            // vertical transport on the bottom face of level k
            const double div = double(U10) - double(U00) + (double(V01) - double(V00));
            Wc = Wc + div;
            const bool mw = (k >= 1) && (Kc >= kwet + 1);  // layers k-1 and k both wet
            sWm[tid] = mw ? R(Wc) : R(0);
        }
        __syncthreads();

        // ---- assembly for the cells of the tile ----
        const R Wm_b = sWm[tid];
        if (cell) {
            const int c = tid, cw = tid - 1, cs = tid - TX;
            const long long o = idx3(S, pi, pj, k);

            // vertical fluxes through the bottom face (between levels k-1 and k)
            R fzT_bot = R(0), fzu_bot = R(0), fzv_bot = R(0);
            R E_bot = R(0);
            if (k >= 1) {
                if (Wm_b != R(0)) {
                    // reconstruct the full temperature from differences relative to the
                    // upwind cell (anomaly steps plus reference-profile steps)
                    const bool pos = Wm_b > R(0);
                    const int kc = pos ? k - 1 : k;
                    const R ta = pos ? wt[5] : wt[0], tb = pos ? wt[4] : wt[1], tcv = pos ? wt[3] : wt[2];
                    const R td = pos ? wt[2] : wt[3], te = pos ? wt[1] : wt[4];
                    const int la = pos ? k - 3 : k + 2, lb = pos ? k - 2 : k + 1;
                    const int ld = pos ? k : k - 1, le = pos ? k + 1 : k - 2;
                    auto okl = [&](int l) { return l >= 0 && l < nz && Kc >= nz - l; };
                    const R da = (ta - tcv) + (pos ? dtr[kc * 4 + 0] : dtr[kc * 4 + 3]);
                    const R db = (tb - tcv) + (pos ? dtr[kc * 4 + 1] : dtr[kc * 4 + 2]);
                    const R dd = (td - tcv) + (pos ? dtr[kc * 4 + 2] : dtr[kc * 4 + 1]);
                    const R de = (te - tcv) + (pos ? dtr[kc * 4 + 3] : dtr[kc * 4 + 0]);
                    const R rel = recon(da, db, R(0), dd, de, okl(la), okl(lb), true, okl(ld), okl(le));
                    fzT_bot = Wm_b * (tcv + rel);
                    // reference profile carried through this face, relative to tref(k)
                    E_bot = pos ? Wm_b * (-dtr[k * 4 + 1]) : R(0);
                }
                const R Fu = R(0.5) * (sWm[cw] + Wm_b);
                if (Fu != R(0)) {
                    R pu[6];
                    bool oku[6];
#pragma unroll
                    for (int r = 0; r < 6; ++r) {
                        const int l = k - 3 + r;
                        pu[r] = wu[5 - r];
                        oku[r] = (l >= 0 && l < nz && Ku >= nz - l);
                    }
                    fzu_bot = upwind_flux(Fu, pu, oku);
                }
                const R Fv = R(0.5) * (sWm[cs] + Wm_b);
                if (Fv != R(0)) {
                    R pv[6];
                    bool okv[6];
#pragma unroll
                    for (int r = 0; r < 6; ++r) {
                        const int l = k - 3 + r;
                        pv[r] = wv[5 - r];
                        okv[r] = (l >= 0 && l < nz && Kv >= nz - l);
                    }
                    fzv_bot = upwind_flux(Fv, pv, okv);
                }
            }

            // tracer
            R GT = R(0);
            if (Kc >= kwet) {
                const R vol = area * dzk;
                R E_top;
                if (k == nz - 1) {
                    E_top = R(Wsurf) * R(S.tref[k]);  // volume flux through the surface, full T
                } else {
                    // upwind cell k+1 when the face transport is downward
                    E_top = (Wm_top > R(0)) ? R(0) : Wm_top * (-dtr[k * 4 + 2]);
                }
                const R divF = (fxT[c] - fxT[cw]) + (fyT[c] - fyT[cs]) + (fzT_top - fzT_bot);
                GT = (-divF + (E_top - E_bot)) / vol;
                if (k == nz - 1) GT += (tstar - wt[2]) * rinv;
            }
            // u momentum
            R GUm = R(0);
            if (Ku >= kwet) {
                const R vol = area * dzk;
                const R divF = (fxu[c] - fxu[cw]) + (fyu[c] - fyu[cs]) + (fzu_top - fzu_bot);
                GUm = -divF / vol + (sQv[cw] + sQv[c]) / (R(2) * vol) - (sP[c] - sP[cw]) / dxc;
                if (k == nz - 1) GUm += wind_u;
            }
            // v momentum
            R GVm = R(0);
            if (Kv >= kwet) {
                const R vol = dxv0 * dy * dzk;
                const R divF = (fxv[c] - fxv[cw]) + (fyv[c] - fyv[cs]) + (fzv_top - fzv_bot);
                GVm = -divF / vol - (sQu[cs] + sQu[c]) / (R(2) * vol) - (sP[c] - sP[cs]) / dy;
                if (k == nz - 1) GVm += wind_v;
            }

            // AB2 predictor; G^n replaces G^{n-1}
            R* gtp = f3<R>(S.gt);
            R* gup = f3<R>(S.gu);
            R* gvp = f3<R>(S.gv);
            const R hT = c_new * GT - c_old * gtp[o];
            const R hU = c_new * GUm - c_old * gup[o];
            const R hV = c_new * GVm - c_old * gvp[o];
            gtp[o] = GT;
            gup[o] = GUm;
            gvp[o] = GVm;
            f3<R>(S.ts)[o] = wt[2] + dt * hT;
            f3<R>(S.us)[o] = wu[2] + dt * hU;
            f3<R>(S.vs)[o] = wv[2] + dt * hV;
            if (Ku >= kwet) gUacc += double(S.dz[k]) * double(hU);
            if (Kv >= kwet) gVacc += double(S.dz[k]) * double(hV);

            fzT_top = fzT_bot;
            fzu_top = fzu_bot;
            fzv_top = fzv_bot;
        }
        Wm_top = Wm_b;
        __syncthreads();
    }
    if (cell) {
        S.gU[idx2(S, pi, pj)] = gUacc;
        S.gV[idx2(S, pi, pj)] = gVacc;
    }
}

template <typename R>
hipError_t launch_tendency(const DevState& s, int first, hipStream_t st) {
    dim3 block(TX, TY);
    dim3 grid((s.nx + TX - 2) / (TX - 1), (s.ny + TY - 2) / (TY - 1));
    hipLaunchKernelGGL(k_tend<R>, grid, block, 0, st, s, first);
    return hipGetLastError();
}

template hipError_t launch_tendency<double>(const DevState&, int, hipStream_t);
template hipError_t launch_tendency<float>(const DevState&, int, hipStream_t);

}  // namespace ocn
