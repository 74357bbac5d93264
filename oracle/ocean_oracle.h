/*
 * ocean_oracle.h -- declarations of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library; the product library never includes,
 * links or calls it. It shares no header, helper or table with the GPU path.
 *
 * The oracle advances a hydrostatic Boussinesq ocean on an Arakawa C-grid by
 * one explicit baroclinic step followed by the sub-cycled split-explicit
 * barotropic loop (paper Sec. 5.2 "New numerical methods" and Sec. 5.3
 * "Optimization of ocean free surface dynamics"). Everything is double
 * precision, plain loops, no blocking or fusion.
 */
#ifndef OCEAN_ORACLE_H
#define OCEAN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Grid, physical constants and time-stepping parameters in one flat record. */
typedef struct orc_desc {
    int32_t nx, ny, nz;            /* interior cells; k = 0 is the bottom layer   */
    int32_t periodic_x, periodic_y;/* 1 = periodic, 0 = bounded by walls          */
    int32_t coords;                /* 0 = Cartesian beta-plane, 1 = lat-lon sphere */
    int32_t n_substeps;            /* barotropic substeps per baroclinic step     */
    int32_t salinity;              /* 1: salinity S is carried and the equation of
                                      state is the nonlinear eos_* form; 0: T only,
                                      linear in T with alpha                      */
    double x0, y0, dx, dy;         /* Cartesian: metres. lat-lon: lon0, lat_south, dlon, dlat in degrees */
    double f0, beta;               /* beta-plane Coriolis f = f0 + beta (y - Ly/2) */
    double radius, omega;          /* sphere radius (m) and rotation rate (1/s)   */
    double dt, chi;                /* baroclinic step (s) and AB2 offset          */
    double g, alpha, rho0, t_ref;  /* gravity, thermal expansion, density, EOS reference T */
    double kappa;                  /* vertical diffusivity = viscosity (m^2/s)    */
    double restore_tau;            /* surface restoring time (s); <= 0 turns it off */
    double pgf_weight;             /* epsilon: the pressure gradient of the momentum step is
                                      taken from T^n + epsilon dt Ghat_T (0..1)            */
    /* equation of state with salinity (density anomaly in kg/m^3, z the depth in
     * m, Ta = T - eos_t0, Sa = S - eos_s0):
     * rho' = -a0 (1 + lambda1 Ta / 2 + mu1 z) Ta + b0 (1 - lambda2 Sa / 2 - mu2 z) Sa - nu Ta Sa */
    double eos_a0, eos_b0, eos_lambda1, eos_lambda2, eos_mu1, eos_mu2, eos_nu, eos_t0, eos_s0;
    int32_t momentum_form;         /* 0: flux form; 1: vector-invariant form       */
    int32_t reserved;
} orc_desc;

typedef struct orc_model orc_model;

/* Field identifiers for orc_set_field / orc_get_field. 3D fields are [k][j][i]
 * (nz*ny*nx), 2D fields [j][i] (ny*nx); W is (nz+1)*ny*nx on z-faces. */
enum {
    ORC_U = 0, ORC_V = 1, ORC_T = 2, ORC_ETA = 3, ORC_UBT = 4, ORC_VBT = 5,
    ORC_ETA_MEAN = 6, ORC_UBT_MEAN = 7, ORC_VBT_MEAN = 8, ORC_W = 9,
    ORC_GU_PREV = 10, ORC_GV_PREV = 11, ORC_GT_PREV = 12,
    ORC_TAUX = 13, ORC_TAUY = 14, ORC_TSTAR = 15, ORC_P = 16,
    ORC_KAPPA = 17,  /* z-face diffusivity, nz*ny*nx, slot k = face between layers k-1 and k;
                        setting NULL returns to the constant */
    ORC_VISC = 18,   /* z-face momentum coefficient on tracer faces (get only): the viscosity
                        of Richardson-number mixing, else the diffusivity */
    ORC_U_PRED = 19, ORC_V_PRED = 20, ORC_T_PRED = 21,  /* AB2-predicted u*, v*, T* */
    ORC_GU_SLOW = 22, ORC_GV_SLOW = 23,                 /* barotropic slow forcing (m^2/s^2) */
    ORC_S = 24, ORC_GS_PREV = 25,                       /* salinity (g/kg) and its AB2 history */
    ORC_SSTAR = 26, ORC_S_PRED = 27                     /* surface restoring salinity; predicted S* */
};

/* Stages of one step, in order (orc_run_stage): the diffusivity diagnosis of
 * convective or Richardson-number mixing; tendencies, AB2 predictor and slow
 * forcing; barotropic substeps; implicit vertical diffusion and depth-mean
 * correction. orc_step runs all four and then advances the step count, the
 * time and the AB2 start flag; orc_run_stage does not. */
enum { ORC_STAGE_MIXING = 0, ORC_STAGE_TENDENCY = 1, ORC_STAGE_BAROTROPIC = 2, ORC_STAGE_COLUMN = 3 };

/* Tendency term selectors for orc_eval_tendencies. */
enum { ORC_TERM_ADV = 1, ORC_TERM_COR = 2, ORC_TERM_PGF = 4, ORC_TERM_WIND = 8,
       ORC_TERM_RESTORE = 16, ORC_TERM_ALL = 31 };

/* Number of doubles written by orc_diagnostics. */
#define ORC_NDIAG 18

orc_model* orc_create(const orc_desc* d, const double* dz, const int32_t* kbottom);
void       orc_destroy(orc_model* m);
int        orc_set_field(orc_model* m, int field, const double* src);
int        orc_get_field(orc_model* m, int field, double* dst);
void       orc_set_first_step(orc_model* m, int first);
/* Convective adjustment: with kappa_conv > 0 every step starts by setting the
 * face diffusivity to kappa_conv where N^2 < 0 and to the constant elsewhere
 * (it replaces a prescribed field); kappa_conv <= 0 returns to the constant. */
void       orc_set_convective(orc_model* m, double kappa_conv);
/* Richardson-number mixing: with nu0 > 0 every step starts by diagnosing the
 * face viscosity (u, v) and diffusivity (T) from the current state,
 * Pacanowski-Philander form with constants nu0, alpha, nub, kappab and conv
 * where N^2 < 0 (see richardson_faces); nu0 <= 0 returns to the constant.
 * Replaces convective adjustment and any prescribed field. */
void       orc_set_richardson(orc_model* m, double nu0, double alpha, double nub, double kappab, double conv);
int        orc_get_first_step(const orc_model* m);
void       orc_step(orc_model* m, int n);
int        orc_run_stage(orc_model* m, int stage);
void       orc_diagnostics(const orc_model* m, double* out);

/* Stage-level entry points used by the physics and unit pins. */
/* gs (salinity tendency) may be NULL; it is written only when salinity is on. */
void   orc_eval_tendencies(const orc_model* m, int terms, double* gu, double* gv, double* gt, double* gs);
/* Buoyancy b = -g rho'/rho0 of water with temperature T and salinity S at depth
 * z (m, positive down) under the model's equation of state (S ignored when
 * salinity is off, where b = g alpha (T - t_ref)). */
double orc_buoyancy(const orc_model* m, double T, double S, double z);
double orc_weno5z(double a, double b, double c, double d, double e);
double orc_weno3(double b, double c, double d);
double orc_reconstruct(const double* s, const int32_t* ok);
void   orc_thomas(int n, const double* a, const double* b, const double* c,
                  const double* d, double* x);
double orc_neumaier_sum(const double* x, int64_t n);
void   orc_column_zflux(int nz, const double* phi, const int32_t* wet,
                        const double* wface, double* flux);

/* Closure inputs and outputs (see ocean_oracle.c for the feature order). */
int    orc_closure_features(const orc_model* m, int din, const double* mean, const double* std, double* X);
void   orc_closure_kappa(const orc_model* m, const double* Y, double kappa0, double* kw);

/* Closure network (mlp_oracle.c): row-major matrices, X n x din, W1 din x h1,
 * W2 h1 x h2, W3 h2 x dout; Y = relu(relu(X W1 + b1) W2 + b2) W3 + b3. */
void   orc_mlp_forward(const double* X, int n, int din, int h1, int h2, int dout, const double* W1,
                       const double* b1, const double* W2, const double* b2, const double* W3, const double* b3,
                       double* H1, double* H2, double* Y);
double orc_mlp_backward(const double* X, const double* T, int n, int din, int h1, int h2, int dout,
                        const double* W1, const double* b1, const double* W2, const double* b2, const double* W3,
                        const double* b3, double* gW1, double* gb1, double* gW2, double* gb2, double* gW3,
                        double* gb3);
void   orc_adam(double* p, const double* g, double* m, double* v, int64_t n, int t, double lr, double beta1,
                double beta2, double eps);

#ifdef __cplusplus
}
#endif
#endif
