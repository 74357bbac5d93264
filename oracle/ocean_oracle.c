/*
 * ocean_oracle.c -- plain FP64 CPU oracle of one split-explicit hydrostatic step.
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU-baseline
 * leg of the benchmark are its only users; the product path never links it and
 * it shares no code with the GPU kernels.
 *
 * The paper (Sec. 5.2) names the scheme classes: hydrostatic Boussinesq
 * equations in finite volume on a staggered Arakawa C-grid, implicit-explicit
 * second-order Adams-Bashforth time stepping, vertically implicit diffusion by
 * backward Euler with a tridiagonal solve, and WENO advection of momentum and
 * tracers. Sec. 5.3 adds the split-explicit free surface: the depth-averaged
 * barotropic mode is sub-cycled explicitly inside each baroclinic step. Sec. 5.1
 * says the tendencies depend on two diagnostics only, hydrostatic pressure and
 * vertical diffusivity. The paper gives no formulas; every detail it leaves
 * open is fixed below in a comment that states the reading taken.
 *
 * Layout: 3D arrays are [k][j][i] with k = 0 the bottom layer, 2D arrays [j][i].
 * Staggering: T at cell centres, u on west faces x_{i-1/2}, v on south faces
 * y_{j-1/2}, W on bottom faces z_{k-1/2} (face index 0..nz), eta/U/V likewise
 * in 2D. Every sum over k runs bottom to top. Compile with -ffp-contract=off.
 */
#include "ocean_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define WENO_EPS 1e-8
#define PI 3.14159265358979323846
#define DEG2RAD (PI / 180.0)

struct orc_model {
    orc_desc d;
    int nx, ny, nz;
    double* dz;          /* nz layer thicknesses, bottom to top */
    int32_t* kb;         /* nx*ny number of wet layers, counted from the surface */
    double *u, *v, *T;   /* prognostic 3D state */
    double *eta, *U, *V; /* barotropic state: free surface (m), depth-integrated velocity (m^2/s) */
    double *gu_prev, *gv_prev, *gt_prev;      /* AB2 history */
    double *eta_mean, *U_mean, *V_mean;       /* substep averages of the last step */
    double *us, *vs, *ts;                     /* AB2-predicted u*, v*, T* (tendency stage output) */
    double *S, *gs_prev, *sstar, *ss;         /* salinity, its AB2 history, restoring target, S* */
    double* zc;                               /* depth of each layer centre (m, positive down) */
    double *gU, *gV;                          /* barotropic slow forcing (tendency stage output) */
    double *taux, *tauy, *tstar;              /* surface forcing (N/m^2, N/m^2, degC) */
    double *kw;          /* prescribed diffusivity on z-faces (m^2/s), or NULL for the constant */
    double *kvw;         /* viscosity on z-faces for u and v, or NULL: they then use kw */
    double kappa_conv;   /* > 0: convective adjustment, kappa_conv on faces with N^2 < 0 */
    int ri_on;           /* Richardson-number mixing (orc_set_richardson) */
    double ri_nu0, ri_alpha, ri_nub, ri_kappab, ri_conv;
    int first_step;
    int64_t step;
    double time;
};

/* ------------------------------------------------------------------------- */
/* Grid geometry (Sec. 5.2: finite volume on a C-grid; Sec. 6: lat-lon domain) */

static double rad(double deg) { return deg * DEG2RAD; }

static double lat_centre(const orc_model* m, int j) { return m->d.y0 + (j + 0.5) * m->d.dy; }
static double lat_south(const orc_model* m, int j) { return m->d.y0 + j * m->d.dy; }

/* x-distance between centres i-1 and i along row j (also the u control-volume width) */
static double dx_c(const orc_model* m, int j) {
    if (m->d.coords == 0) return m->d.dx;
    return m->d.radius * cos(rad(lat_centre(m, j))) * rad(m->d.dx);
}
/* length of the south face of cell (i,j), where v lives */
static double dx_v(const orc_model* m, int j) {
    if (m->d.coords == 0) return m->d.dx;
    return m->d.radius * cos(rad(lat_south(m, j))) * rad(m->d.dx);
}
static double dy_m(const orc_model* m) {
    if (m->d.coords == 0) return m->d.dy;
    return m->d.radius * rad(m->d.dy);
}
static double area_c(const orc_model* m, int j) { return dx_c(m, j) * dy_m(m); }
static double coriolis_c(const orc_model* m, int j) {
    if (m->d.coords == 0) {
        double ly = m->ny * m->d.dy;
        return m->d.f0 + m->d.beta * ((j + 0.5) * m->d.dy - 0.5 * ly);
    }
    return 2.0 * m->d.omega * sin(rad(lat_centre(m, j)));
}
/* Coriolis parameter on the south face of row j (where v lives) */
static double coriolis_s(const orc_model* m, int j) {
    if (m->d.coords == 0) {
        double ly = m->ny * m->d.dy;
        return m->d.f0 + m->d.beta * (j * m->d.dy - 0.5 * ly);
    }
    return 2.0 * m->d.omega * sin(rad(lat_south(m, j)));
}
/* spherical metric factor tan(phi)/a; zero on the beta-plane */
static double metric_c(const orc_model* m, int j) {
    if (m->d.coords == 0) return 0.0;
    return tan(rad(lat_centre(m, j))) / m->d.radius;
}

/* ------------------------------------------------------------------------- */
/* Index maps, masks and guarded accessors. Periodic directions wrap; cells
 * beyond a bounded wall are land and read as zero. */

static int map_i(const orc_model* m, int i) {
    if (i >= 0 && i < m->nx) return i;
    if (m->d.periodic_x) { int r = i % m->nx; return r < 0 ? r + m->nx : r; }
    return -1;
}
static int map_j(const orc_model* m, int j) {
    if (j >= 0 && j < m->ny) return j;
    if (m->d.periodic_y) { int r = j % m->ny; return r < 0 ? r + m->ny : r; }
    return -1;
}
static int cell_wet(const orc_model* m, int i, int j, int k) {
    if (k < 0 || k >= m->nz) return 0;
    int ii = map_i(m, i), jj = map_j(m, j);
    if (ii < 0 || jj < 0) return 0;
    return k >= m->nz - m->kb[jj * m->nx + ii];
}
static int u_wet(const orc_model* m, int i, int j, int k) { return cell_wet(m, i - 1, j, k) && cell_wet(m, i, j, k); }
static int v_wet(const orc_model* m, int i, int j, int k) { return cell_wet(m, i, j - 1, k) && cell_wet(m, i, j, k); }
/* interior z-face k (between layers k-1 and k) with water on both sides */
static int w_wet(const orc_model* m, int i, int j, int k) {
    return k >= 1 && k <= m->nz - 1 && cell_wet(m, i, j, k - 1) && cell_wet(m, i, j, k);
}
static double at3(const orc_model* m, const double* f, int i, int j, int k) {
    if (k < 0 || k >= m->nz) return 0.0;
    int ii = map_i(m, i), jj = map_j(m, j);
    if (ii < 0 || jj < 0) return 0.0;
    return f[((size_t)k * m->ny + jj) * m->nx + ii];
}
static double at2(const orc_model* m, const double* f, int i, int j) {
    int ii = map_i(m, i), jj = map_j(m, j);
    if (ii < 0 || jj < 0) return 0.0;
    return f[(size_t)jj * m->nx + ii];
}
static double atw(const orc_model* m, const double* w3, int i, int j, int kf) {
    int ii = map_i(m, i), jj = map_j(m, j);
    if (ii < 0 || jj < 0 || kf < 0 || kf > m->nz) return 0.0;
    return w3[((size_t)kf * m->ny + jj) * m->nx + ii];
}
static size_t id3(const orc_model* m, int i, int j, int k) { return ((size_t)k * m->ny + j) * m->nx + i; }
static size_t id2(const orc_model* m, int i, int j) { return (size_t)j * m->nx + i; }

/* volume transports through the faces of cell (i,j,k), m^3/s */
static double U3(const orc_model* m, const double* u, int i, int j, int k) {
    return u_wet(m, i, j, k) ? at3(m, u, i, j, k) * dy_m(m) * m->dz[k] : 0.0;
}
static double V3(const orc_model* m, const double* v, int i, int j, int k) {
    return v_wet(m, i, j, k) ? at3(m, v, i, j, k) * dx_v(m, j) * m->dz[k] : 0.0;
}
static double depth_u(const orc_model* m, int i, int j) {
    double h = 0.0;
    for (int k = 0; k < m->nz; ++k) if (u_wet(m, i, j, k)) h += m->dz[k];
    return h;
}
static double depth_v(const orc_model* m, int i, int j) {
    double h = 0.0;
    for (int k = 0; k < m->nz; ++k) if (v_wet(m, i, j, k)) h += m->dz[k];
    return h;
}

/* ------------------------------------------------------------------------- */
/* WENO reconstructions (Sec. 5.2 names WENO for momentum and tracers; its
 * weights are not printed). Reading: fifth-order WENO-Z (Borges et al. 2008,
 * exponent 2, eps = 1e-8) with the Jiang-Shu smoothness indicators, reduced to
 * third-order WENO-JS and then to first-order upwind where the five-point
 * stencil touches land or a wall ("adaptive order", Sec. 5.2).
 * The face lies between c and d; c is the upwind cell. */

double orc_weno5z(double a, double b, double c, double d, double e) {
    double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
    double s0 = a - 2.0 * b + c, r0 = a - 4.0 * b + 3.0 * c;
    double s1 = b - 2.0 * c + d, r1 = b - d;
    double s2 = c - 2.0 * d + e, r2 = 3.0 * c - 4.0 * d + e;
    double beta0 = 13.0 / 12.0 * s0 * s0 + 0.25 * r0 * r0;
    double beta1 = 13.0 / 12.0 * s1 * s1 + 0.25 * r1 * r1;
    double beta2 = 13.0 / 12.0 * s2 * s2 + 0.25 * r2 * r2;
    double tau = fabs(beta0 - beta2);
    double z0 = tau / (beta0 + WENO_EPS), z1 = tau / (beta1 + WENO_EPS), z2 = tau / (beta2 + WENO_EPS);
    double a0 = 0.1 * (1.0 + z0 * z0);
    double a1 = 0.6 * (1.0 + z1 * z1);
    double a2 = 0.3 * (1.0 + z2 * z2);
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

double orc_weno3(double b, double c, double d) {
    double q0 = (-b + 3.0 * c) / 2.0;
    double q1 = (c + d) / 2.0;
    double beta0 = (c - b) * (c - b);
    double beta1 = (d - c) * (d - c);
    double a0 = (1.0 / 3.0) / ((beta0 + WENO_EPS) * (beta0 + WENO_EPS));
    double a1 = (2.0 / 3.0) / ((beta1 + WENO_EPS) * (beta1 + WENO_EPS));
    return (a0 * q0 + a1 * q1) / (a0 + a1);
}

/* s = (a,b,c,d,e) ordered from far upwind to far downwind; ok flags each point */
double orc_reconstruct(const double* s, const int32_t* ok) {
    if (ok[0] && ok[1] && ok[2] && ok[3] && ok[4]) return orc_weno5z(s[0], s[1], s[2], s[3], s[4]);
    if (ok[1] && ok[2] && ok[3]) return orc_weno3(s[1], s[2], s[3]);
    return s[2];
}

/* Advective flux F*phi_face through a face. p[0..5] are the values at the six
 * points -3..+2 around the face (the face lies between points -1 and 0). For
 * F >= 0 the upwind cell is point -1, else point 0. A zero transport gives a
 * zero flux. */
static double upwind_flux(double F, const double* p, const int32_t* ok) {
    if (F == 0.0) return 0.0;
    double s[5];
    int32_t o[5];
    if (F > 0.0) {
        for (int r = 0; r < 5; ++r) { s[r] = p[r]; o[r] = ok[r]; }
    } else {
        for (int r = 0; r < 5; ++r) { s[r] = p[5 - r]; o[r] = ok[5 - r]; }
    }
    return F * orc_reconstruct(s, o);
}

/* Flux through every z-face 0..nz of one column: wface holds the masked vertical
 * transport at each face, wet flags the layers. Used for tracers and momentum. */
static double column_face_flux(int nz, const double* phi, const int32_t* wet, int kf, double F) {
    double p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) {
        int k = kf - 3 + r;
        int in = (k >= 0 && k < nz);
        p[r] = in ? phi[k] : 0.0;
        ok[r] = in ? wet[k] : 0;
    }
    return upwind_flux(F, p, ok);
}

void orc_column_zflux(int nz, const double* phi, const int32_t* wet, const double* wface, double* flux) {
    for (int kf = 0; kf <= nz; ++kf) flux[kf] = column_face_flux(nz, phi, wet, kf, wface[kf]);
}

/* ------------------------------------------------------------------------- */
/* Tridiagonal solve by Thomas elimination: sub-diagonal a (coupling to k-1),
 * diagonal b, super-diagonal c (coupling to k+1); eliminate upward, substitute
 * downward. No pivoting: the backward-Euler matrices are diagonally dominant. */
void orc_thomas(int n, const double* a, const double* b, const double* c, const double* d, double* x) {
    double* cp = (double*)malloc(sizeof(double) * (size_t)n);
    double* dp = (double*)malloc(sizeof(double) * (size_t)n);
    cp[0] = c[0] / b[0];
    dp[0] = d[0] / b[0];
    for (int k = 1; k < n; ++k) {
        double den = b[k] - a[k] * cp[k - 1];
        cp[k] = c[k] / den;
        dp[k] = (d[k] - a[k] * dp[k - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int k = n - 2; k >= 0; --k) x[k] = dp[k] - cp[k] * x[k + 1];
    free(cp);
    free(dp);
}

/* Compensated (Neumaier) summation in index order. */
double orc_neumaier_sum(const double* x, int64_t n) {
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) comp += (s - t) + x[i];
        else comp += (x[i] - t) + s;
        s = t;
    }
    return s + comp;
}

/* ------------------------------------------------------------------------- */
/* Diagnostics shared by the tendency: vertical transport and pressure. */

/* Vertical transport W (m^3/s) on every z-face from continuity, integrated
 * upward from zero at the bottom. The surface value is not used as an
 * advective flux: reading of a linear free surface with fixed cell volumes. */
static void compute_w(const orc_model* m, const double* u, const double* v, double* w3) {
    for (int j = 0; j < m->ny; ++j)
        for (int i = 0; i < m->nx; ++i) {
            double w = 0.0;
            w3[id2(m, i, j)] = 0.0;
            for (int k = 0; k < m->nz; ++k) {
                double div = U3(m, u, i + 1, j, k) - U3(m, u, i, j, k) + V3(m, v, i, j + 1, k) - V3(m, v, i, j, k);
                w = w - div;
                w3[((size_t)(k + 1) * m->ny + j) * m->nx + i] = w;
            }
        }
}

/* Equation of state. Temperature only (the benchmarked configurations): a
 * linear buoyancy b = g alpha (T - t_ref). With salinity (reading: the paper's
 * realistic runs carry heat and salt, Sec. 6, and name no equation of state;
 * the simplified seawater equation of state of Roquet et al. 2015 is taken):
 * the density anomaly rho' = -a0 (1 + lambda1 Ta/2 + mu1 z) Ta
 * + b0 (1 - lambda2 Sa/2 - mu2 z) Sa - nu Ta Sa with Ta = T - t0, Sa = S - s0
 * and z the depth, quadratic in T and S (cabbeling) with pressure-dependent
 * expansion coefficients (thermobaricity), and b = -g rho' / rho0. */
double orc_buoyancy(const orc_model* m, double T, double S, double z) {
    const orc_desc* d = &m->d;
    if (!d->salinity) return d->g * d->alpha * (T - d->t_ref);
    const double ta = T - d->eos_t0, sa = S - d->eos_s0;
    const double rho = -d->eos_a0 * (1.0 + 0.5 * d->eos_lambda1 * ta + d->eos_mu1 * z) * ta
                     + d->eos_b0 * (1.0 - 0.5 * d->eos_lambda2 * sa - d->eos_mu2 * z) * sa
                     - d->eos_nu * ta * sa;
    return -d->g * rho / d->rho0;
}

/* buoyancy of cell (i, j, k) at its own depth */
static double cell_b(const orc_model* m, const double* T, const double* S, int i, int j, int k) {
    const size_t c = id3(m, i, j, k);
    return orc_buoyancy(m, T[c], S ? S[c] : 0.0, m->zc[k]);
}

/* Squared buoyancy frequency on the interior face below layer k: the buoyancy
 * difference of the two layers, both taken at the face's depth (with the
 * linear equation of state g alpha (T_k - T_{k-1})), over the centre spacing. */
static double face_n2(const orc_model* m, const double* T, const double* S, int i, int j, int k) {
    const double dzc = 0.5 * (m->dz[k - 1] + m->dz[k]);
    const size_t c = id3(m, i, j, k), b = id3(m, i, j, k - 1);
    if (!m->d.salinity) return m->d.g * m->d.alpha * (T[c] - T[b]) / dzc;
    const double zf = m->zc[k] + 0.5 * m->dz[k];
    return (orc_buoyancy(m, T[c], S[c], zf) - orc_buoyancy(m, T[b], S[b], zf)) / dzc;
}

/* Hydrostatic kinematic pressure p with dp/dz = b and p = 0 at the rigid-lid
 * surface z = 0 (the surface-elevation part of the pressure lives in the
 * barotropic mode). Integrated downward: half the top layer with the top
 * buoyancy, then the trapezoid rule between adjacent layer centres (centre
 * spacing times the mean buoyancy). This is the first of the two 3D
 * diagnostics of Sec. 5.1. S is ignored (and may be NULL) without salinity. */
static void compute_p(const orc_model* m, const double* T, const double* S, double* p) {
    for (int j = 0; j < m->ny; ++j)
        for (int i = 0; i < m->nx; ++i) {
            double pk = 0.0;
            for (int k = m->nz - 1; k >= 0; --k) {
                if (!cell_wet(m, i, j, k)) { p[id3(m, i, j, k)] = 0.0; continue; }
                double bk = cell_b(m, T, S, i, j, k);
                if (k == m->nz - 1) {
                    pk = -0.5 * m->dz[k] * bk;
                } else {
                    double bk1 = cell_b(m, T, S, i, j, k + 1);
                    double dzc = 0.5 * (m->dz[k] + m->dz[k + 1]);
                    pk = pk - dzc * 0.5 * (bk + bk1);
                }
                p[id3(m, i, j, k)] = pk;
            }
        }
}

/* Pressure-gradient accelerations along z-levels at a u point (west face of
 * cell i) and a v point (south face of cell j): minus the difference of the
 * kinematic pressure of the two cells over their centre distance. */
static double pgf_u(const orc_model* m, const double* p, int i, int j, int k) {
    return -(at3(m, p, i, j, k) - at3(m, p, i - 1, j, k)) / dx_c(m, j);
}
static double pgf_v(const orc_model* m, const double* p, int i, int j, int k) {
    return -(at3(m, p, i, j, k) - at3(m, p, i, j - 1, k)) / dy_m(m);
}

/* ------------------------------------------------------------------------- */
/* Advective fluxes (flux form, WENO face values). */

static double wmask(const orc_model* m, const double* w3, int i, int j, int kf) {
    return w_wet(m, i, j, kf) ? atw(m, w3, i, j, kf) : 0.0;
}

/* tracer through the west face of cell (i,j,k) */
static double tracer_xflux(const orc_model* m, const double* u, const double* T, int i, int j, int k) {
    double F = U3(m, u, i, j, k), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, T, i - 3 + r, j, k); ok[r] = cell_wet(m, i - 3 + r, j, k); }
    return upwind_flux(F, p, ok);
}
static double tracer_yflux(const orc_model* m, const double* v, const double* T, int i, int j, int k) {
    double F = V3(m, v, i, j, k), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, T, i, j - 3 + r, k); ok[r] = cell_wet(m, i, j - 3 + r, k); }
    return upwind_flux(F, p, ok);
}
static double tracer_zflux(const orc_model* m, const double* w3, const double* T, int i, int j, int kf) {
    double F = wmask(m, w3, i, j, kf), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, T, i, j, kf - 3 + r); ok[r] = cell_wet(m, i, j, kf - 3 + r); }
    return upwind_flux(F, p, ok);
}

/* Momentum in flux form (reading: the paper does not state the momentum
 * advection form; flux form with the spherical metric term carried by the
 * Coriolis operator). Transports are averaged to the faces of the u and v
 * control volumes; u and v values are reconstructed by the same WENO rule,
 * with a masked velocity point counting as invalid. */

/* u through the centre of cell (ic,j): between u(ic) and u(ic+1) */
static double u_xflux(const orc_model* m, const double* u, int ic, int j, int k) {
    double F = 0.5 * (U3(m, u, ic, j, k) + U3(m, u, ic + 1, j, k)), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, u, ic - 2 + r, j, k); ok[r] = u_wet(m, ic - 2 + r, j, k); }
    return upwind_flux(F, p, ok);
}
/* u through the corner (i-1/2, jf-1/2): between u(i,jf-1) and u(i,jf) */
static double u_yflux(const orc_model* m, const double* u, const double* v, int i, int jf, int k) {
    double F = 0.5 * (V3(m, v, i - 1, jf, k) + V3(m, v, i, jf, k)), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, u, i, jf - 3 + r, k); ok[r] = u_wet(m, i, jf - 3 + r, k); }
    return upwind_flux(F, p, ok);
}
static double u_zflux(const orc_model* m, const double* u, const double* w3, int i, int j, int kf) {
    double F = 0.5 * (wmask(m, w3, i - 1, j, kf) + wmask(m, w3, i, j, kf)), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, u, i, j, kf - 3 + r); ok[r] = u_wet(m, i, j, kf - 3 + r); }
    return upwind_flux(F, p, ok);
}
/* v through the centre of cell (i,jc): between v(jc) and v(jc+1) */
static double v_yflux(const orc_model* m, const double* v, int i, int jc, int k) {
    double F = 0.5 * (V3(m, v, i, jc, k) + V3(m, v, i, jc + 1, k)), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, v, i, jc - 2 + r, k); ok[r] = v_wet(m, i, jc - 2 + r, k); }
    return upwind_flux(F, p, ok);
}
/* v through the corner (if-1/2, j-1/2): between v(if-1,j) and v(if,j) */
static double v_xflux(const orc_model* m, const double* u, const double* v, int iF, int j, int k) {
    double F = 0.5 * (U3(m, u, iF, j - 1, k) + U3(m, u, iF, j, k)), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, v, iF - 3 + r, j, k); ok[r] = v_wet(m, iF - 3 + r, j, k); }
    return upwind_flux(F, p, ok);
}
static double v_zflux(const orc_model* m, const double* v, const double* w3, int i, int j, int kf) {
    double F = 0.5 * (wmask(m, w3, i, j - 1, kf) + wmask(m, w3, i, j, kf)), p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) { p[r] = at3(m, v, i, j, kf - 3 + r); ok[r] = v_wet(m, i, j, kf - 3 + r); }
    return upwind_flux(F, p, ok);
}

/* Coriolis (reading: energy-conserving C-grid form). Each wet cell carries
 * Q = f~ V_c with f~ = f + u_c tan(phi)/a, the metric term of the momentum
 * equations on the sphere; u gets the average of Q v_c over its two cells,
 * v minus the average of Q u_c. Summed against u V_u and v V_v the two terms
 * cancel exactly. */
static double cell_Q(const orc_model* m, const double* u, int i, int j, int k) {
    if (!cell_wet(m, i, j, k)) return 0.0;
    int jj = map_j(m, j);
    double uc = 0.5 * (at3(m, u, i, j, k) + at3(m, u, i + 1, j, k));
    double ft = coriolis_c(m, jj) + metric_c(m, jj) * uc;
    return ft * area_c(m, jj) * m->dz[k];
}
static double cell_vbar(const orc_model* m, const double* v, int i, int j, int k) {
    return 0.5 * (at3(m, v, i, j, k) + at3(m, v, i, j + 1, k));
}
static double cell_ubar(const orc_model* m, const double* u, int i, int j, int k) {
    return 0.5 * (at3(m, u, i, j, k) + at3(m, u, i + 1, j, k));
}

/* Momentum in vector-invariant form (paper Sec. 5.2 names WENO momentum
 * advection on curvilinear grids, after Silvestri et al.; this form is a
 * reading). The advection and Coriolis terms of (u.grad)u + f k x u are
 * written as (f + zeta) k x u + grad(|u|^2 / 2) + w du/dz:
 *  - zeta is the relative vorticity at a cell corner, the circulation of u, v
 *    around it over its area (on the sphere this carries the metric term),
 *    and 0 at a corner that touches land (free slip);
 *  - at a u point, zeta is reconstructed along y from the six corners of its
 *    column by the WENO rule (order reduced where corners touch land),
 *    upwind of vbar, the mean of the four surrounding v, on zeta / ZETA_REF:
 *    WENO's epsilon (1e-8) is absolute, and vorticity of order 1e-5 1/s
 *    would leave every smoothness indicator far below it, so that the
 *    weights would stay linear; in units of a typical Coriolis parameter
 *    they act as they do on order-one data; the term is
 *    (f + zeta) vbar with f at the u point's latitude; a v point likewise
 *    reconstructs zeta along x upwind of ubar and takes -(f + zeta) ubar;
 *  - the kinetic energy K = (u_w^2 + u_e^2 + v_s^2 + v_n^2) / 4 lives at cell
 *    centres and its difference over the centre distance gives the gradient;
 *  - w du/dz is the vertical flux divergence of the flux form minus u times
 *    the divergence of the vertical transport of the velocity's control
 *    volume.
 * The Coriolis part f vbar (f ubar) counts as ORC_TERM_COR, the rest as
 * ORC_TERM_ADV. */
#define ZETA_REF 1e-4
static double uvel(const orc_model* m, const double* u, int i, int j, int k) {
    return u_wet(m, i, j, k) ? at3(m, u, i, j, k) : 0.0;
}
static double vvel(const orc_model* m, const double* v, int i, int j, int k) {
    return v_wet(m, i, j, k) ? at3(m, v, i, j, k) : 0.0;
}
/* corner (i-1/2, j-1/2): water in all four cells around it */
static int corner_wet(const orc_model* m, int i, int j, int k) {
    return cell_wet(m, i - 1, j - 1, k) && cell_wet(m, i, j - 1, k) && cell_wet(m, i - 1, j, k) && cell_wet(m, i, j, k);
}
static double corner_zeta(const orc_model* m, const double* u, const double* v, int i, int j, int k) {
    if (!corner_wet(m, i, j, k)) return 0.0;
    const int jj = map_j(m, j), js = map_j(m, j - 1);
    const double dy = dy_m(m);
    const double circ = dy * (vvel(m, v, i, j, k) - vvel(m, v, i - 1, j, k))
                      - (dx_c(m, jj) * uvel(m, u, i, j, k) - dx_c(m, js) * uvel(m, u, i, j - 1, k));
    return circ / (dx_v(m, jj) * dy);
}
static double cell_ke(const orc_model* m, const double* u, const double* v, int i, int j, int k) {
    const double uw = uvel(m, u, i, j, k), ue = uvel(m, u, i + 1, j, k);
    const double vs = vvel(m, v, i, j, k), vn = vvel(m, v, i, j + 1, k);
    return 0.25 * (uw * uw + ue * ue) + 0.25 * (vs * vs + vn * vn);
}
/* upwind reconstruction of the value between points 2 and 3 of p[0..5] */
static double upwind_value(double F, const double* p, const int32_t* ok) {
    double s[5];
    int32_t o[5];
    if (F > 0.0) {
        for (int r = 0; r < 5; ++r) { s[r] = p[r]; o[r] = ok[r]; }
    } else {
        for (int r = 0; r < 5; ++r) { s[r] = p[5 - r]; o[r] = ok[5 - r]; }
    }
    return orc_reconstruct(s, o);
}
/* u point (i, j): advection (ADV) and Coriolis (COR) parts of the vector-invariant form */
static void vi_u(const orc_model* m, const double* u, const double* v, const double* w3, int i, int j, int k,
                 double* adv, double* cor) {
    const double vbar = 0.25 * (vvel(m, v, i - 1, j, k) + vvel(m, v, i - 1, j + 1, k) + vvel(m, v, i, j, k)
                                + vvel(m, v, i, j + 1, k));
    double p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) {
        p[r] = corner_zeta(m, u, v, i, j - 2 + r, k) / ZETA_REF;
        ok[r] = corner_wet(m, i, j - 2 + r, k);
    }
    const double zeta = ZETA_REF * upwind_value(vbar, p, ok);
    const int jj = map_j(m, j);
    const double vol = area_c(m, jj) * m->dz[k];
    const double ke = -(cell_ke(m, u, v, i, j, k) - cell_ke(m, u, v, i - 1, j, k)) / dx_c(m, jj);
    const double wt = 0.5 * (wmask(m, w3, i - 1, j, k + 1) + wmask(m, w3, i, j, k + 1));
    const double wb = 0.5 * (wmask(m, w3, i - 1, j, k) + wmask(m, w3, i, j, k));
    const double vert = ((u_zflux(m, u, w3, i, j, k + 1) - u_zflux(m, u, w3, i, j, k))
                         - uvel(m, u, i, j, k) * (wt - wb)) / vol;
    *adv = zeta * vbar + ke - vert;
    *cor = coriolis_c(m, jj) * vbar;
}
/* v point (i, j) */
static void vi_v(const orc_model* m, const double* u, const double* v, const double* w3, int i, int j, int k,
                 double* adv, double* cor) {
    const double ubar = 0.25 * (uvel(m, u, i, j - 1, k) + uvel(m, u, i + 1, j - 1, k) + uvel(m, u, i, j, k)
                                + uvel(m, u, i + 1, j, k));
    double p[6];
    int32_t ok[6];
    for (int r = 0; r < 6; ++r) {
        p[r] = corner_zeta(m, u, v, i - 2 + r, j, k) / ZETA_REF;
        ok[r] = corner_wet(m, i - 2 + r, j, k);
    }
    const double zeta = ZETA_REF * upwind_value(ubar, p, ok);
    const int jj = map_j(m, j);
    const double dy = dy_m(m);
    const double vol = dx_v(m, jj) * dy * m->dz[k];
    const double ke = -(cell_ke(m, u, v, i, j, k) - cell_ke(m, u, v, i, j - 1, k)) / dy;
    const double wt = 0.5 * (wmask(m, w3, i, j - 1, k + 1) + wmask(m, w3, i, j, k + 1));
    const double wb = 0.5 * (wmask(m, w3, i, j - 1, k) + wmask(m, w3, i, j, k));
    const double vert = ((v_zflux(m, v, w3, i, j, k + 1) - v_zflux(m, v, w3, i, j, k))
                         - vvel(m, v, i, j, k) * (wt - wb)) / vol;
    *adv = -zeta * ubar + ke - vert;
    *cor = -coriolis_s(m, jj) * ubar;
}

/* Tendency of a tracer (T or S) in a wet cell: flux-form advection and, in
 * the top layer, restoring towards the target field. */
static double tracer_tendency(const orc_model* m, int terms, const double* q, const double* qstar,
                              const double* w3, int i, int j, int k) {
    double g = 0.0;
    if (!cell_wet(m, i, j, k)) return 0.0;
    const double vol = area_c(m, j) * m->dz[k];
    if (terms & ORC_TERM_ADV) {
        double div = tracer_xflux(m, m->u, q, i + 1, j, k) - tracer_xflux(m, m->u, q, i, j, k)
                   + tracer_yflux(m, m->v, q, i, j + 1, k) - tracer_yflux(m, m->v, q, i, j, k)
                   + tracer_zflux(m, w3, q, i, j, k + 1) - tracer_zflux(m, w3, q, i, j, k);
        g += -div / vol;
    }
    if ((terms & ORC_TERM_RESTORE) && k == m->nz - 1 && m->d.restore_tau > 0.0)
        g += (qstar[id2(m, i, j)] - q[id3(m, i, j, k)]) / m->d.restore_tau;
    return g;
}

void orc_eval_tendencies(const orc_model* m, int terms, double* gu, double* gv, double* gt, double* gs) {
    const size_t n3 = (size_t)m->nx * m->ny * m->nz;
    const size_t nf = (size_t)m->nx * m->ny * (m->nz + 1);
    double* w3 = (double*)calloc(nf, sizeof(double));
    double* p = (double*)calloc(n3, sizeof(double));
    compute_w(m, m->u, m->v, w3);
    compute_p(m, m->T, m->S, p);
    const double* u = m->u;
    const double* v = m->v;
    const double* T = m->T;
    const double dy = dy_m(m);
    const int top = m->nz - 1;

    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                const size_t c = id3(m, i, j, k);
                const double dz = m->dz[k];
                /* tracers */
                gt[c] = tracer_tendency(m, terms, T, m->tstar, w3, i, j, k);
                if (gs && m->d.salinity) gs[c] = tracer_tendency(m, terms, m->S, m->sstar, w3, i, j, k);
                double g;
                /* u momentum */
                g = 0.0;
                if (u_wet(m, i, j, k) && m->d.momentum_form == 1) {
                    double adv, cor;
                    vi_u(m, u, v, w3, i, j, k, &adv, &cor);
                    if (terms & ORC_TERM_ADV) g += adv;
                    if (terms & ORC_TERM_COR) g += cor;
                    if (terms & ORC_TERM_PGF) g += pgf_u(m, p, i, j, k);
                    if ((terms & ORC_TERM_WIND) && k == top)
                        g += m->taux[id2(m, i, j)] / (m->d.rho0 * dz);
                } else if (u_wet(m, i, j, k)) {
                    double vol = area_c(m, j) * dz;
                    if (terms & ORC_TERM_ADV) {
                        double div = u_xflux(m, u, i, j, k) - u_xflux(m, u, i - 1, j, k)
                                   + u_yflux(m, u, v, i, j + 1, k) - u_yflux(m, u, v, i, j, k)
                                   + u_zflux(m, u, w3, i, j, k + 1) - u_zflux(m, u, w3, i, j, k);
                        g += -div / vol;
                    }
                    if (terms & ORC_TERM_COR)
                        g += (cell_Q(m, u, i - 1, j, k) * cell_vbar(m, v, i - 1, j, k)
                              + cell_Q(m, u, i, j, k) * cell_vbar(m, v, i, j, k)) / (2.0 * vol);
                    if (terms & ORC_TERM_PGF) g += pgf_u(m, p, i, j, k);
                    if ((terms & ORC_TERM_WIND) && k == top)
                        g += m->taux[id2(m, i, j)] / (m->d.rho0 * dz);
                }
                gu[c] = g;
                /* v momentum */
                g = 0.0;
                if (v_wet(m, i, j, k) && m->d.momentum_form == 1) {
                    double adv, cor;
                    vi_v(m, u, v, w3, i, j, k, &adv, &cor);
                    if (terms & ORC_TERM_ADV) g += adv;
                    if (terms & ORC_TERM_COR) g += cor;
                    if (terms & ORC_TERM_PGF) g += pgf_v(m, p, i, j, k);
                    if ((terms & ORC_TERM_WIND) && k == top)
                        g += m->tauy[id2(m, i, j)] / (m->d.rho0 * dz);
                } else if (v_wet(m, i, j, k)) {
                    double vol = dx_v(m, j) * dy * dz;
                    if (terms & ORC_TERM_ADV) {
                        double div = v_xflux(m, u, v, i + 1, j, k) - v_xflux(m, u, v, i, j, k)
                                   + v_yflux(m, v, i, j, k) - v_yflux(m, v, i, j - 1, k)
                                   + v_zflux(m, v, w3, i, j, k + 1) - v_zflux(m, v, w3, i, j, k);
                        g += -div / vol;
                    }
                    if (terms & ORC_TERM_COR)
                        g += -(cell_Q(m, u, i, j - 1, k) * cell_ubar(m, u, i, j - 1, k)
                               + cell_Q(m, u, i, j, k) * cell_ubar(m, u, i, j, k)) / (2.0 * vol);
                    if (terms & ORC_TERM_PGF) g += pgf_v(m, p, i, j, k);
                    if ((terms & ORC_TERM_WIND) && k == top)
                        g += m->tauy[id2(m, i, j)] / (m->d.rho0 * dz);
                }
                gv[c] = g;
            }
    free(w3);
    free(p);
}

/* ------------------------------------------------------------------------- */
/* Backward-Euler vertical diffusion of one column (Sec. 5.2: vertically
 * implicit diffusion, backward Euler, tridiagonal solver). Face diffusivities:
 * kappa (the constant, or the prescribed face field) on interior wet faces of
 * the tracer column; momentum takes the mean of the two neighbouring
 * tracer-face values on faces wet for that velocity point (reading: the same
 * diffusivity acts on T, u and v, unit Prandtl number). Zero flux at the bottom and
 * at the surface, so the column integral sum dz*phi is preserved. kind: 0 T,
 * 1 u, 2 v. */
static double tracer_face_kappa(const orc_model* m, int i, int j, int kf) {
    if (!w_wet(m, i, j, kf)) return 0.0;
    return m->kw ? at3(m, m->kw, i, j, kf) : m->d.kappa;
}
/* momentum coefficient on a tracer face: the viscosity field when one is set
 * (Richardson-number mixing), else the diffusivity */
static double tracer_face_visc(const orc_model* m, int i, int j, int kf) {
    if (!m->kvw) return tracer_face_kappa(m, i, j, kf);
    if (!w_wet(m, i, j, kf)) return 0.0;
    return at3(m, m->kvw, i, j, kf);
}
static double face_kappa(const orc_model* m, int kind, int i, int j, int kf) {
    if (kf <= 0 || kf >= m->nz) return 0.0;
    if (kind == 0) return tracer_face_kappa(m, i, j, kf);
    if (kind == 1) {
        if (!(u_wet(m, i, j, kf) && u_wet(m, i, j, kf - 1))) return 0.0;
        return 0.5 * (tracer_face_visc(m, i - 1, j, kf) + tracer_face_visc(m, i, j, kf));
    }
    if (!(v_wet(m, i, j, kf) && v_wet(m, i, j, kf - 1))) return 0.0;
    return 0.5 * (tracer_face_visc(m, i, j - 1, kf) + tracer_face_visc(m, i, j, kf));
}

/* Richardson-number vertical mixing (Sec. 6 runs a Richardson-number-based
 * parameterization of shear and convective mixing; it gives no formula, so
 * the Pacanowski-Philander (1981) form is the reading). On an interior wet
 * face k of column (i, j), from the state at the start of the step:
 *   N^2 = g alpha (T_k - T_{k-1}) / dzc_k (with salinity, the buoyancy
 *         difference of the two layers at the face's depth over dzc_k),
 *   S^2 = ((uc_k - uc_{k-1})^2 + (vc_k - vc_{k-1})^2) / dzc_k^2, with uc, vc
 *         the velocities averaged to the cell centre (a dry or closed-edge
 *         face counts as 0),
 *   N^2 < 0: viscosity = diffusivity = conv (convective turbulence);
 *   else Ri = N^2 / max(S^2, 1e-16), r = 1 / (1 + a Ri),
 *        viscosity nu = nu0 r^2 + nub, diffusivity kappa = nu r + kappab.
 * Dry faces and face 0 take 0. */
static void richardson_faces(orc_model* m) {
    const int nx = m->nx, ny = m->ny, nz = m->nz;
    const size_t n3 = (size_t)nx * ny * nz;
    if (!m->kw) m->kw = (double*)malloc(sizeof(double) * n3);
    if (!m->kvw) m->kvw = (double*)malloc(sizeof(double) * n3);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double kap = 0.0, nu = 0.0;
                if (k >= 1 && w_wet(m, i, j, k)) {
                    const int ie = (i + 1 < nx) ? i + 1 : (m->d.periodic_x ? 0 : -1);
                    const int jn = (j + 1 < ny) ? j + 1 : (m->d.periodic_y ? 0 : -1);
                    double uc[2], vc[2];
                    for (int q = 0; q < 2; ++q) {
                        const int kk = k - 1 + q;
                        const double ue = ie >= 0 ? m->u[id3(m, ie, j, kk)] : 0.0;
                        const double vn = jn >= 0 ? m->v[id3(m, i, jn, kk)] : 0.0;
                        uc[q] = 0.5 * (m->u[id3(m, i, j, kk)] + ue);
                        vc[q] = 0.5 * (m->v[id3(m, i, j, kk)] + vn);
                    }
                    const double dzc = 0.5 * (m->dz[k - 1] + m->dz[k]);
                    const double n2 = face_n2(m, m->T, m->S, i, j, k);
                    const double du = uc[1] - uc[0], dv = vc[1] - vc[0];
                    const double s2 = (du * du + dv * dv) / (dzc * dzc);
                    if (n2 < 0.0) {
                        kap = m->ri_conv;
                        nu = m->ri_conv;
                    } else {
                        const double ri = n2 / fmax(s2, 1e-16);
                        const double r = 1.0 / (1.0 + m->ri_alpha * ri);
                        nu = m->ri_nu0 * r * r + m->ri_nub;
                        kap = nu * r + m->ri_kappab;
                    }
                }
                m->kw[id3(m, i, j, k)] = kap;
                m->kvw[id3(m, i, j, k)] = nu;
            }
}

static void implicit_column(const orc_model* m, int kind, int i, int j, const double* phistar, double* out) {
    const int nz = m->nz;
    const double dt = m->d.dt;
    double* a = (double*)calloc((size_t)nz * 5, sizeof(double));
    double *b = a + nz, *c = b + nz, *d = c + nz, *x = d + nz;
    for (int k = 0; k < nz; ++k) {
        double klo = face_kappa(m, kind, i, j, k);
        double khi = face_kappa(m, kind, i, j, k + 1);
        double lo = (k >= 1) ? dt * klo / (0.5 * (m->dz[k - 1] + m->dz[k])) : 0.0;
        double hi = (k <= nz - 2) ? dt * khi / (0.5 * (m->dz[k] + m->dz[k + 1])) : 0.0;
        a[k] = -lo;
        c[k] = -hi;
        b[k] = m->dz[k] + lo + hi;
        d[k] = m->dz[k] * phistar[id3(m, i, j, k)];
    }
    orc_thomas(nz, a, b, c, d, x);
    for (int k = 0; k < nz; ++k) out[id3(m, i, j, k)] = x[k];
    free(a);
}

/* ------------------------------------------------------------------------- */
/* One baroclinic step followed by the barotropic substeps. Stage order
 * (reading of the time-stepping sequence of Fig. 2, whose image is missing):
 * diffusivity diagnosis -> diagnostics w and p -> tendencies -> AB2 predictor
 * and barotropic slow forcing -> substeps -> implicit vertical diffusion and
 * depth-mean correction. The implicit diffusion of the predicted fields does
 * not depend on the substeps, so it runs beside the correction that needs
 * them. Each stage is also callable on its own (orc_run_stage). */

/* Stage 0: the face diffusivity of convective adjustment or Richardson-number
 * mixing, diagnosed from the state at the start of the step (Sec. 5.1: the
 * diffusivity is a diagnostic of the current state). Nothing with the
 * constant or a prescribed field. */
static void stage_mixing(orc_model* m) {
    const int nx = m->nx, ny = m->ny, nz = m->nz;
    const size_t n3 = (size_t)nx * ny * nz;
    /* convective adjustment: kappa_conv on interior wet faces where the water
     * above is denser than the water below (N^2 = g alpha dT/dz < 0), the
     * constant elsewhere */
    if (m->ri_on) richardson_faces(m);
    else if (m->kappa_conv > 0.0) {
        if (!m->kw) m->kw = (double*)malloc(sizeof(double) * n3);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    double kap = 0.0;
                    if (w_wet(m, i, j, k)) {
                        const int unstable = m->d.salinity ? face_n2(m, m->T, m->S, i, j, k) < 0.0
                                                           : m->T[id3(m, i, j, k)] < m->T[id3(m, i, j, k - 1)];
                        kap = unstable ? m->kappa_conv : m->d.kappa;
                    }
                    m->kw[id3(m, i, j, k)] = kap;
                }
    }
}

/* Stage 1: tendencies, AB2 predictor (u*, v*, T*, new histories) and the
 * barotropic slow forcing. */
static void stage_tendency(orc_model* m) {
    const int nx = m->nx, ny = m->ny, nz = m->nz;
    const size_t n3 = (size_t)nx * ny * nz;
    const double dt = m->d.dt, chi = m->d.chi, eps = m->d.pgf_weight;
    double* tfb = (double*)malloc(sizeof(double) * n3);
    double* pfb = (double*)malloc(sizeof(double) * n3);
    double* gu = (double*)malloc(sizeof(double) * n3);
    double* gv = (double*)malloc(sizeof(double) * n3);
    double* gt = (double*)malloc(sizeof(double) * n3);
    double* gs = m->d.salinity ? (double*)malloc(sizeof(double) * n3) : NULL;
    double* sfb = m->d.salinity ? (double*)malloc(sizeof(double) * n3) : NULL;

    /* tendencies G^n of the current state: advection, Coriolis, wind and
     * restoring; the baroclinic pressure gradient is added below */
    orc_eval_tendencies(m, ORC_TERM_ALL & ~ORC_TERM_PGF, gu, gv, gt, gs);

    /* AB2 predictor: Ghat = (3/2+chi) G^n - (1/2+chi) G^{n-1}; forward Euler on
     * the first step (reading of the "second-order Adams-Bashforth" start).
     * The tracer goes first: T* = T^n + dt Ghat_T. */
    for (size_t c = 0; c < n3; ++c) {
        const double ht = m->first_step ? gt[c] : (1.5 + chi) * gt[c] - (0.5 + chi) * m->gt_prev[c];
        m->ts[c] = m->T[c] + dt * ht;
        tfb[c] = m->T[c] + eps * dt * ht;
        m->gt_prev[c] = gt[c];
        if (gs) {  /* salinity likewise */
            const double hs = m->first_step ? gs[c] : (1.5 + chi) * gs[c] - (0.5 + chi) * m->gs_prev[c];
            m->ss[c] = m->S[c] + dt * hs;
            sfb[c] = m->S[c] + eps * dt * hs;
            m->gs_prev[c] = gs[c];
        }
    }

    /* Forward-backward pressure gradient (reading of the implicit-explicit AB2
     * of Sec. 5.2 for the internal gravity waves): the momentum step takes the
     * hydrostatic pressure of T^n + epsilon dt Ghat_T, the tracer just
     * predicted weighted by epsilon, instead of extrapolating the pressure
     * gradient of past states. AB2 alone amplifies oscillations whose
     * frequency times dt exceeds about 0.5, which internal waves on converging
     * meridians reach at the benchmarked resolutions; with epsilon = 3/4 the
     * coupled pair stays damped up to about 1.3. The AB2 history of u and v
     * holds their other terms only. */
    compute_p(m, tfb, sfb, pfb);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = id3(m, i, j, k);
                double hu = m->first_step ? gu[c] : (1.5 + chi) * gu[c] - (0.5 + chi) * m->gu_prev[c];
                double hv = m->first_step ? gv[c] : (1.5 + chi) * gv[c] - (0.5 + chi) * m->gv_prev[c];
                m->gu_prev[c] = gu[c];
                m->gv_prev[c] = gv[c];
                if (u_wet(m, i, j, k)) hu += pgf_u(m, pfb, i, j, k);
                if (v_wet(m, i, j, k)) hv += pgf_v(m, pfb, i, j, k);
                m->us[c] = m->u[c] + dt * hu;
                m->vs[c] = m->v[c] + dt * hv;
                gu[c] = hu;  /* keep Ghat for the barotropic slow forcing */
                gv[c] = hv;
            }

    /* barotropic slow forcing: depth integral of the AB2 momentum tendency */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double su = 0.0, sv = 0.0;
            for (int k = 0; k < nz; ++k) {
                if (u_wet(m, i, j, k)) su += m->dz[k] * gu[id3(m, i, j, k)];
                if (v_wet(m, i, j, k)) sv += m->dz[k] * gv[id3(m, i, j, k)];
            }
            m->gU[id2(m, i, j)] = su;
            m->gV[id2(m, i, j)] = sv;
        }
    free(tfb); free(pfb); free(gu); free(gv); free(gt); free(gs); free(sfb);
}

/* Stage 2: barotropic substeps (Sec. 5.3: explicit sub-cycling of the 2D
 * mode). Reading: forward-backward, free surface first, then transports from
 * the new surface gradient plus the slow forcing, dtau = dt/Ns. The substeps
 * run on to t^n + 3dt/2 (M = Ns + Ns/2 of them); the new eta, U, V are the
 * averages of eta^q, U^q, V^q (q = 1..M) with weights a_q proportional to
 * cos^2(pi t), t = q/Ns - 1, |t| < 1/2, a window centred on t^{n+1}; the
 * transport that moves the free surface over the step is
 * Ubar = sum_l A_l U^l / Ns with A_l = sum_{q>l} a_q, so that
 * eta^{n+1} - eta^n = -dt div Ubar exactly. */
static void stage_barotropic(orc_model* m) {
    const int nx = m->nx, ny = m->ny;
    const size_t n2 = (size_t)nx * ny;
    const int ns = m->d.n_substeps, M = ns + ns / 2;
    const double dt = m->d.dt, dtau = dt / ns, g = m->d.g, dy = dy_m(m);
    double* en = (double*)malloc(sizeof(double) * n2);
    double* Un = (double*)malloc(sizeof(double) * n2);
    double* Vn = (double*)malloc(sizeof(double) * n2);
    double* Hu = (double*)malloc(sizeof(double) * n2);
    double* Hv = (double*)malloc(sizeof(double) * n2);
    double* sU = (double*)calloc(n2, sizeof(double));   /* sum_l A_l U^l */
    double* sV = (double*)calloc(n2, sizeof(double));
    double* fE = (double*)calloc(n2, sizeof(double));   /* sum_q a_q eta^q */
    double* fU = (double*)calloc(n2, sizeof(double));
    double* fV = (double*)calloc(n2, sizeof(double));
    double* a = (double*)calloc((size_t)M + 1, sizeof(double));
    double asum = 0.0;
    for (int q = 1; q <= M; ++q) {
        const double t = (double)q / ns - 1.0;
        const double c = fabs(t) < 0.5 ? cos(PI * t) : 0.0;
        a[q] = c * c;
        asum += a[q];
    }
    for (int q = 1; q <= M; ++q) a[q] /= asum;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) { Hu[id2(m, i, j)] = depth_u(m, i, j); Hv[id2(m, i, j)] = depth_v(m, i, j); }
    for (int l = 0; l < M; ++l) {
        double Al = 0.0;
        for (int q = l + 1; q <= M; ++q) Al += a[q];
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double div = dy * (at2(m, m->U, i + 1, j) - at2(m, m->U, i, j))
                           + dx_v(m, j + 1) * at2(m, m->V, i, j + 1) - dx_v(m, j) * at2(m, m->V, i, j);
                en[id2(m, i, j)] = m->eta[id2(m, i, j)] - dtau / area_c(m, j) * div;
                sU[id2(m, i, j)] += Al * m->U[id2(m, i, j)];
                sV[id2(m, i, j)] += Al * m->V[id2(m, i, j)];
            }
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = id2(m, i, j);
                double hu = Hu[c], hv = Hv[c];
                Un[c] = hu > 0.0 ? m->U[c] + dtau * (-g * hu * (en[c] - at2(m, en, i - 1, j)) / dx_c(m, j) + m->gU[c]) : 0.0;
                Vn[c] = hv > 0.0 ? m->V[c] + dtau * (-g * hv * (en[c] - at2(m, en, i, j - 1)) / dy + m->gV[c]) : 0.0;
            }
        for (size_t c = 0; c < n2; ++c) {
            m->eta[c] = en[c];
            m->U[c] = Un[c];
            m->V[c] = Vn[c];
            fE[c] += a[l + 1] * en[c];
            fU[c] += a[l + 1] * Un[c];
            fV[c] += a[l + 1] * Vn[c];
        }
    }
    for (size_t c = 0; c < n2; ++c) {
        m->eta[c] = fE[c];
        m->U[c] = fU[c];
        m->V[c] = fV[c];
        m->eta_mean[c] = fE[c];
        m->U_mean[c] = sU[c] / ns;
        m->V_mean[c] = sV[c] / ns;
    }
    free(en); free(Un); free(Vn); free(Hu); free(Hv); free(sU); free(sV); free(fE); free(fU); free(fV); free(a);
}

/* Stage 3: implicit vertical diffusion of the predicted fields, then the
 * depth-mean correction: the depth mean of u** is replaced by Ubar/H, the
 * transport that moved the free surface over the step, so
 * sum dz u^{n+1} = Ubar exactly. */
static void stage_column(orc_model* m) {
    const int nx = m->nx, ny = m->ny, nz = m->nz;
    const size_t n3 = (size_t)nx * ny * nz;
    double* uss = (double*)malloc(sizeof(double) * n3);
    double* vss = (double*)malloc(sizeof(double) * n3);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            implicit_column(m, 0, i, j, m->ts, m->T);
            if (m->d.salinity) implicit_column(m, 0, i, j, m->ss, m->S);
            implicit_column(m, 1, i, j, m->us, uss);
            implicit_column(m, 2, i, j, m->vs, vss);
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t c2 = id2(m, i, j);
            const double hu = depth_u(m, i, j), hv = depth_v(m, i, j);
            double su = 0.0, sv = 0.0;
            for (int k = 0; k < nz; ++k) {
                if (u_wet(m, i, j, k)) su += m->dz[k] * uss[id3(m, i, j, k)];
                if (v_wet(m, i, j, k)) sv += m->dz[k] * vss[id3(m, i, j, k)];
            }
            for (int k = 0; k < nz; ++k) {
                size_t c = id3(m, i, j, k);
                m->u[c] = (hu > 0.0 && u_wet(m, i, j, k)) ? uss[c] + (m->U_mean[c2] - su) / hu : 0.0;
                m->v[c] = (hv > 0.0 && v_wet(m, i, j, k)) ? vss[c] + (m->V_mean[c2] - sv) / hv : 0.0;
            }
        }
    free(uss); free(vss);
}

int orc_run_stage(orc_model* m, int stage) {
    switch (stage) {
    case ORC_STAGE_MIXING: stage_mixing(m); return 0;
    case ORC_STAGE_TENDENCY: stage_tendency(m); return 0;
    case ORC_STAGE_BAROTROPIC: stage_barotropic(m); return 0;
    case ORC_STAGE_COLUMN: stage_column(m); return 0;
    default: return -1;
    }
}

static void step_once(orc_model* m) {
    stage_mixing(m);
    stage_tendency(m);
    stage_barotropic(m);
    stage_column(m);
    m->first_step = 0;
    m->step += 1;
    m->time += m->d.dt;
}

void orc_step(orc_model* m, int n) {
    for (int s = 0; s < n; ++s) step_once(m);
}

/* ------------------------------------------------------------------------- */
/* Diagnostics: compensated sums in (k, j, i) order.
 * out[0] step, [1] time, [2] tracer content sum V_c T, [3] volume sum A eta,
 * [4] mean-volume sum A eta_mean, [5] kinetic energy 1/2 sum (V_u u^2 + V_v v^2),
 * [6] max|u|, [7] max|v|, [8] max|w| on interior wet faces, [9] T min, [10] T max
 * (wet cells), [11] eta min, [12] eta max (wet columns), [13] non-finite count,
 * [14] advective CFL max(|u| dt/dx, |v| dt/dy, |w| dt/dz_c), [15] sum of A_c
 * over wet columns, [16] barotropic CFL of a substep max sqrt(g H) dtau
 * sqrt(1/dx^2 + 1/dy^2) over wet columns, [17] salt content sum V_c S (0
 * without salinity); [13] counts cells with a non-finite u, v, T (or S) and
 * columns with a non-finite eta, U or V. */
void orc_diagnostics(const orc_model* m, double* out) {
    const int nx = m->nx, ny = m->ny, nz = m->nz;
    const size_t n3 = (size_t)nx * ny * nz, n2 = (size_t)nx * ny;
    double* buf = (double*)malloc(sizeof(double) * (n3 > n2 ? n3 : n2));
    double* w3 = (double*)calloc((size_t)nx * ny * (nz + 1), sizeof(double));
    compute_w(m, m->u, m->v, w3);
    const double dt = m->d.dt, dy = dy_m(m);
    size_t n = 0;
    double tmin = INFINITY, tmax = -INFINITY, emin = INFINITY, emax = -INFINITY;
    double umax = 0, vmax = 0, wmax = 0, cfl = 0, nonfinite = 0;

    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = id3(m, i, j, k);
                if (!isfinite(m->u[c]) || !isfinite(m->v[c]) || !isfinite(m->T[c]) ||
                    (m->d.salinity && !isfinite(m->S[c])))
                    nonfinite += 1;
                if (cell_wet(m, i, j, k)) {
                    buf[n++] = area_c(m, j) * m->dz[k] * m->T[c];
                    if (m->T[c] < tmin) tmin = m->T[c];
                    if (m->T[c] > tmax) tmax = m->T[c];
                }
            }
    out[2] = orc_neumaier_sum(buf, (int64_t)n);
    n = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = id3(m, i, j, k);
                double ke = 0.0;
                if (u_wet(m, i, j, k)) {
                    ke += area_c(m, j) * m->dz[k] * m->u[c] * m->u[c];
                    double a = fabs(m->u[c]);
                    if (a > umax) umax = a;
                    if (a * dt / dx_c(m, j) > cfl) cfl = a * dt / dx_c(m, j);
                }
                if (v_wet(m, i, j, k)) {
                    ke += dx_v(m, j) * dy * m->dz[k] * m->v[c] * m->v[c];
                    double a = fabs(m->v[c]);
                    if (a > vmax) vmax = a;
                    if (a * dt / dy > cfl) cfl = a * dt / dy;
                }
                buf[n++] = 0.5 * ke;
                if (w_wet(m, i, j, k)) {
                    double a = fabs(w3[((size_t)k * ny + j) * nx + i] / area_c(m, j));
                    if (a > wmax) wmax = a;
                    double dzc = 0.5 * (m->dz[k - 1] + m->dz[k]);
                    if (a * dt / dzc > cfl) cfl = a * dt / dzc;
                }
            }
    out[5] = orc_neumaier_sum(buf, (int64_t)n);
    n = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = id2(m, i, j);
            if (!isfinite(m->eta[c]) || !isfinite(m->U[c]) || !isfinite(m->V[c])) nonfinite += 1;
            if (m->kb[c] > 0) {
                buf[n++] = area_c(m, j) * m->eta[c];
                if (m->eta[c] < emin) emin = m->eta[c];
                if (m->eta[c] > emax) emax = m->eta[c];
            }
        }
    out[3] = orc_neumaier_sum(buf, (int64_t)n);
    n = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            if (m->kb[id2(m, i, j)] > 0) buf[n++] = area_c(m, j) * m->eta_mean[id2(m, i, j)];
    out[4] = orc_neumaier_sum(buf, (int64_t)n);
    n = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            if (m->kb[id2(m, i, j)] > 0) buf[n++] = area_c(m, j);
    out[15] = orc_neumaier_sum(buf, (int64_t)n);
    /* barotropic gravity-wave CFL of a substep: sqrt(g H) dtau sqrt(1/dx^2 + 1/dy^2)
     * over wet columns, H the column's depth */
    double cflbt = 0.0;
    const double dtau = dt / m->d.n_substeps;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int kb = m->kb[id2(m, i, j)];
            if (kb <= 0) continue;
            double hc = 0.0;
            for (int k = nz - kb; k < nz; ++k) hc += m->dz[k];
            const double dxc = dx_c(m, j);
            const double c = sqrt(m->d.g * hc) * dtau * sqrt(1.0 / (dxc * dxc) + 1.0 / (dy * dy));
            if (c > cflbt) cflbt = c;
        }
    out[16] = cflbt;
    /* salt content sum V_c S over wet cells (0 without salinity) */
    n = 0;
    if (m->d.salinity)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    if (cell_wet(m, i, j, k)) buf[n++] = area_c(m, j) * m->dz[k] * m->S[id3(m, i, j, k)];
    out[17] = orc_neumaier_sum(buf, (int64_t)n);

    out[0] = (double)m->step;
    out[1] = m->time;
    out[6] = umax; out[7] = vmax; out[8] = wmax;
    out[9] = tmin; out[10] = tmax; out[11] = emin; out[12] = emax;
    out[13] = nonfinite; out[14] = cfl;
    free(buf);
    free(w3);
}

/* ------------------------------------------------------------------------- */
/* Construction and field access. */

orc_model* orc_create(const orc_desc* d, const double* dz, const int32_t* kbottom) {
    if (!d || !dz || d->nx <= 0 || d->ny <= 0 || d->nz <= 0 || d->n_substeps <= 0) return NULL;
    orc_model* m = (orc_model*)calloc(1, sizeof(orc_model));
    m->d = *d;
    m->nx = d->nx; m->ny = d->ny; m->nz = d->nz;
    const size_t n3 = (size_t)m->nx * m->ny * m->nz, n2 = (size_t)m->nx * m->ny;
    m->dz = (double*)malloc(sizeof(double) * m->nz);
    memcpy(m->dz, dz, sizeof(double) * m->nz);
    m->kb = (int32_t*)malloc(sizeof(int32_t) * n2);
    for (size_t c = 0; c < n2; ++c) {
        int32_t kb = kbottom ? kbottom[c] : m->nz;
        m->kb[c] = kb < 0 ? 0 : (kb > m->nz ? m->nz : kb);
    }
    double** f3[] = {&m->u, &m->v, &m->T, &m->gu_prev, &m->gv_prev, &m->gt_prev, &m->us, &m->vs, &m->ts,
                     &m->S, &m->gs_prev, &m->ss};
    for (size_t q = 0; q < sizeof(f3) / sizeof(f3[0]); ++q) *f3[q] = (double*)calloc(n3, sizeof(double));
    double** f2[] = {&m->eta, &m->U, &m->V, &m->eta_mean, &m->U_mean, &m->V_mean, &m->taux, &m->tauy, &m->tstar,
                     &m->gU, &m->gV, &m->sstar};
    for (size_t q = 0; q < sizeof(f2) / sizeof(f2[0]); ++q) *f2[q] = (double*)calloc(n2, sizeof(double));
    m->zc = (double*)malloc(sizeof(double) * m->nz);
    {
        double depth = 0.0;  /* from the surface down */
        for (int k = m->nz - 1; k >= 0; --k) {
            m->zc[k] = depth + 0.5 * m->dz[k];
            depth += m->dz[k];
        }
    }
    m->first_step = 1;
    return m;
}

void orc_destroy(orc_model* m) {
    if (!m) return;
    double* all[] = {m->dz, m->u, m->v, m->T, m->gu_prev, m->gv_prev, m->gt_prev, m->eta, m->U, m->V,
                     m->eta_mean, m->U_mean, m->V_mean, m->taux, m->tauy, m->tstar, m->kw, m->kvw,
                     m->us, m->vs, m->ts, m->gU, m->gV, m->S, m->gs_prev, m->sstar, m->ss, m->zc};
    for (size_t q = 0; q < sizeof(all) / sizeof(all[0]); ++q) free(all[q]);
    free(m->kb);
    free(m);
}

static double* field_ptr(orc_model* m, int f, size_t* n) {
    const size_t n3 = (size_t)m->nx * m->ny * m->nz, n2 = (size_t)m->nx * m->ny;
    switch (f) {
    case ORC_U: *n = n3; return m->u;
    case ORC_V: *n = n3; return m->v;
    case ORC_T: *n = n3; return m->T;
    case ORC_ETA: *n = n2; return m->eta;
    case ORC_UBT: *n = n2; return m->U;
    case ORC_VBT: *n = n2; return m->V;
    case ORC_ETA_MEAN: *n = n2; return m->eta_mean;
    case ORC_UBT_MEAN: *n = n2; return m->U_mean;
    case ORC_VBT_MEAN: *n = n2; return m->V_mean;
    case ORC_GU_PREV: *n = n3; return m->gu_prev;
    case ORC_GV_PREV: *n = n3; return m->gv_prev;
    case ORC_GT_PREV: *n = n3; return m->gt_prev;
    case ORC_TAUX: *n = n2; return m->taux;
    case ORC_TAUY: *n = n2; return m->tauy;
    case ORC_TSTAR: *n = n2; return m->tstar;
    case ORC_U_PRED: *n = n3; return m->us;
    case ORC_V_PRED: *n = n3; return m->vs;
    case ORC_T_PRED: *n = n3; return m->ts;
    case ORC_GU_SLOW: *n = n2; return m->gU;
    case ORC_GV_SLOW: *n = n2; return m->gV;
    case ORC_S: *n = n3; return m->S;
    case ORC_GS_PREV: *n = n3; return m->gs_prev;
    case ORC_SSTAR: *n = n2; return m->sstar;
    case ORC_S_PRED: *n = n3; return m->ss;
    default: return NULL;
    }
}

/* Setting u or v stores the masked values (a dry velocity point is zero). */
int orc_set_field(orc_model* m, int f, const double* src) {
    size_t n = 0;
    if (f == ORC_KAPPA) {  /* NULL returns to the constant diffusivity */
        const size_t n3 = (size_t)m->nx * m->ny * m->nz;
        if (!src) { free(m->kw); m->kw = NULL; free(m->kvw); m->kvw = NULL; return 0; }
        if (!m->kw) m->kw = (double*)malloc(sizeof(double) * n3);
        memcpy(m->kw, src, sizeof(double) * n3);
        return 0;
    }
    double* p = field_ptr(m, f, &n);
    if (!p || !src) return -1;
    memcpy(p, src, sizeof(double) * n);
    if (f == ORC_U || f == ORC_V)
        for (int k = 0; k < m->nz; ++k)
            for (int j = 0; j < m->ny; ++j)
                for (int i = 0; i < m->nx; ++i) {
                    int wet = (f == ORC_U) ? u_wet(m, i, j, k) : v_wet(m, i, j, k);
                    if (!wet) p[id3(m, i, j, k)] = 0.0;
                }
    return 0;
}

int orc_get_field(orc_model* m, int f, double* dst) {
    if (!dst) return -1;
    if (f == ORC_W) {
        double* w3 = (double*)calloc((size_t)m->nx * m->ny * (m->nz + 1), sizeof(double));
        compute_w(m, m->u, m->v, w3);
        for (int kf = 0; kf <= m->nz; ++kf)
            for (int j = 0; j < m->ny; ++j)
                for (int i = 0; i < m->nx; ++i)
                    dst[((size_t)kf * m->ny + j) * m->nx + i] = w3[((size_t)kf * m->ny + j) * m->nx + i] / area_c(m, j);
        free(w3);
        return 0;
    }
    if (f == ORC_P) {
        compute_p(m, m->T, m->S, dst);
        return 0;
    }
    if (f == ORC_KAPPA) {  /* the tracer diffusivity in use on every face (0 where dry) */
        for (int k = 0; k < m->nz; ++k)
            for (int j = 0; j < m->ny; ++j)
                for (int i = 0; i < m->nx; ++i) dst[id3(m, i, j, k)] = face_kappa(m, 0, i, j, k);
        return 0;
    }
    if (f == ORC_VISC) {  /* the momentum coefficient on every tracer face (0 where dry or face 0) */
        for (int k = 0; k < m->nz; ++k)
            for (int j = 0; j < m->ny; ++j)
                for (int i = 0; i < m->nx; ++i)
                    dst[id3(m, i, j, k)] = (k >= 1 && k < m->nz) ? tracer_face_visc(m, i, j, k) : 0.0;
        return 0;
    }
    size_t n = 0;
    double* p = field_ptr(m, f, &n);
    if (!p) return -1;
    memcpy(dst, p, sizeof(double) * n);
    return 0;
}

void orc_set_first_step(orc_model* m, int first) { m->first_step = first ? 1 : 0; }
void orc_set_convective(orc_model* m, double kappa_conv) {
    m->kappa_conv = kappa_conv > 0.0 ? kappa_conv : 0.0;
    m->ri_on = 0;
    free(m->kvw);
    m->kvw = NULL;
    if (m->kappa_conv == 0.0) { free(m->kw); m->kw = NULL; }
}
void orc_set_richardson(orc_model* m, double nu0, double alpha, double nub, double kappab, double conv) {
    free(m->kvw);
    m->kvw = NULL;
    free(m->kw);
    m->kw = NULL;
    m->kappa_conv = 0.0;
    m->ri_on = nu0 > 0.0;
    m->ri_nu0 = nu0;
    m->ri_alpha = alpha;
    m->ri_nub = nub;
    m->ri_kappab = kappab;
    m->ri_conv = conv;
    if (m->ri_on) richardson_faces(m);
}
int orc_get_first_step(const orc_model* m) { return m->first_step; }

/* ------------------------------------------------------------------------- */
/* Learned-closure plumbing: the per-column input vector of the network and the
 * map from its output to face diffusivities. The paper motivates learned
 * parameterizations (Sec. 3) and runs with a vertical-mixing closure (Sec. 6);
 * the network replaces the diffusivity of the implicit vertical diffusion.
 *
 * Features of column (i, j), in this order (nz = number of layers):
 *   [0, nz)        T at layer centres
 *   [nz, 2nz)      u at centres, mean of the west and east faces
 *   [2nz, 3nz)     v at centres, mean of the south and north faces
 *   [3nz, 4nz)     N^2 on face k (g alpha dT/dz, or from the equation of state
 *                  with salinity; slot k; the bottom face k = 0
 *                  and faces without water on both sides count as dry)
 *   4nz, 4nz+1     wind stress at the centre, means of the two faces' tau_x, tau_y
 *   4nz+2          surface restoring flux dz_top (T* - T_top) / tau (K m/s), 0 when off
 *   [4nz+3, din)   zero padding
 * A wet entry is normalised, (x - mean) / std; dry entries (layers below the
 * sea floor, dry faces, land columns) are 0. X is (ny nx) x din, row j nx + i. */
int orc_closure_features(const orc_model* m, int din, const double* mean, const double* std, double* X) {
    const int nz = m->nz;
    if (din < 4 * nz + 3) return -1;
    for (int j = 0; j < m->ny; ++j)
        for (int i = 0; i < m->nx; ++i) {
            double* x = X + id2(m, i, j) * (size_t)din;
            for (int f = 0; f < din; ++f) x[f] = 0.0;
            const int K = m->kb[id2(m, i, j)];
            if (K == 0) continue;
#define PUT(f, val) x[f] = ((val) - mean[f]) / std[f]
            for (int k = nz - K; k < nz; ++k) {
                PUT(k, at3(m, m->T, i, j, k));
                PUT(nz + k, 0.5 * (at3(m, m->u, i, j, k) + at3(m, m->u, i + 1, j, k)));
                PUT(2 * nz + k, 0.5 * (at3(m, m->v, i, j, k) + at3(m, m->v, i, j + 1, k)));
                if (w_wet(m, i, j, k)) PUT(3 * nz + k, face_n2(m, m->T, m->S, i, j, k));
            }
            PUT(4 * nz, 0.5 * (at2(m, m->taux, i, j) + at2(m, m->taux, i + 1, j)));
            PUT(4 * nz + 1, 0.5 * (at2(m, m->tauy, i, j) + at2(m, m->tauy, i, j + 1)));
            const double q = m->d.restore_tau > 0.0
                                 ? m->dz[nz - 1] * (m->tstar[id2(m, i, j)] - at3(m, m->T, i, j, nz - 1)) / m->d.restore_tau
                                 : 0.0;
            PUT(4 * nz + 2, q);
#undef PUT
        }
    return 0;
}

/* Network output -> face diffusivity. Y is (ny nx) x nz: slot k holds log10
 * of the diffusivity on face k (between layers k-1 and k; slot 0, the bottom
 * face, is unused). A wet interior face takes 10^y clipped to [1e-7, 1] m^2/s,
 * or kappa0 when y is not finite; dry faces take 0. kw is nz x ny x nx like
 * ORC_KAPPA (slot 0 is 0). */
void orc_closure_kappa(const orc_model* m, const double* Y, double kappa0, double* kw) {
    const int nz = m->nz;
    for (int j = 0; j < m->ny; ++j)
        for (int i = 0; i < m->nx; ++i) {
            const double* y = Y + id2(m, i, j) * (size_t)nz;
            for (int k = 0; k < nz; ++k) {
                double v = 0.0;
                if (w_wet(m, i, j, k)) v = isfinite(y[k]) ? fmin(1.0, fmax(1e-7, pow(10.0, y[k]))) : kappa0;
                kw[id3(m, i, j, k)] = v;
            }
        }
}
