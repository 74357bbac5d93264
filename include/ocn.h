/*
 * ocn.h -- C ABI of the MI355X split-explicit hydrostatic ocean step.
 *
 * One explicit baroclinic step of the hydrostatic Boussinesq equations on a
 * finite-volume Arakawa C-grid (WENO advection of tracers and momentum,
 * Coriolis, hydrostatic pressure gradient of a linear equation of state, AB2
 * update, backward-Euler vertical diffusion by a tridiagonal solve per column),
 * followed by the sub-cycled split-explicit barotropic free-surface loop
 * (paper Sec. 5.2 "New numerical methods" and Sec. 5.3 "Optimization of ocean
 * free surface dynamics"). The user sets up a grid (resolution, extent, levels,
 * bathymetry), an initial state and forcing, advances n steps of size dt and
 * reads the state and diagnostics (the problem as stated in paper Sec. 6).
 *
 * Memory and streams. The library never allocates device memory: the caller
 * passes one device arena (for example a torch uint8 tensor on the GPU) whose
 * size ocn_state_arena_bytes reports, and a HIP stream. Every kernel and copy
 * of a state runs on that stream. Host buffers passed to get/set calls belong
 * to the caller and are used only during the call.
 *
 * Errors. Every call returns an ocn_status; no C++ exception crosses the ABI.
 * Invalid arguments return OCN_E_INVALID with no side effect and a message in
 * ocn_last_error(). HIP failures return OCN_E_DEVICE with the HIP error text.
 * ocn_step is asynchronous: a device fault surfaces at the next synchronising
 * call. Handles are not thread-safe; distinct handles are independent.
 *
 * Layout on the host. 3D fields are double [k][j][i] with k = 0 the bottom
 * layer, nz*ny*nx values; 2D fields are double [j][i], ny*nx values. u lives on
 * west faces x_{i-1/2}, v on south faces y_{j-1/2}, T at cell centres; the
 * barotropic U, V are depth-integrated velocities (m^2/s) on the same faces.
 */
#ifndef OCN_H
#define OCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCN_ABI_VERSION 3u

typedef enum {
    OCN_OK = 0,
    OCN_E_INVALID = -1,     /* bad argument; nothing changed                       */
    OCN_E_NOMEM = -2,       /* arena too small or host allocation failed           */
    OCN_E_DEVICE = -3,      /* a HIP call failed                                   */
    OCN_E_UNSTABLE = -4,    /* diagnostics found non-finite values                 */
    OCN_E_STATE = -5,       /* call not allowed in the current state               */
    OCN_E_UNSUPPORTED = -6  /* valid request the library does not implement        */
} ocn_status;

/* Arithmetic of the 3D path. OCN_FP32: tendencies, AB2 and the column solve in
 * FP32 with temperature stored as an anomaly from a per-level FP64 reference
 * profile; the barotropic state, its substeps and averages, the depth sums of
 * the slow forcing and of the correction, and all diagnostics sums stay FP64.
 * (Paper Sec. 2: both 64- and 32-bit runs are measured.) */
typedef enum { OCN_FP64 = 0, OCN_FP32 = 1 } ocn_precision;
typedef enum { OCN_CARTESIAN = 0, OCN_LATLON = 1 } ocn_coords;

typedef struct ocn_grid_desc {
    int32_t nx, ny, nz;       /* interior cells, >= 1 each                          */
    int32_t halo;             /* halo width of the padded layout, 3..8              */
    int32_t periodic_x;       /* 1 periodic, 0 walls                                */
    int32_t periodic_y;       /* 1 periodic (Cartesian only), 0 walls               */
    int32_t coords;           /* ocn_coords                                         */
    int32_t reserved;         /* must be 0                                          */
    double x0, y0, dx, dy;    /* Cartesian: m (x0, y0 unused). lat-lon: degrees:
                                 west edge, south edge, dlon, dlat                  */
    double f0, beta;          /* beta-plane Coriolis f = f0 + beta (y - Ly/2)       */
    double radius, omega;     /* sphere radius (m), rotation rate (1/s)             */
    const double* dz;         /* nz layer thicknesses (m), bottom to top; required  */
    const int32_t* kbottom;   /* ny*nx wet layers per column counted from the surface
                                 (0 = land); NULL = every column full depth         */
} ocn_grid_desc;

typedef struct ocn_params {
    int32_t precision;        /* ocn_precision                                      */
    int32_t n_substeps;       /* barotropic substeps per step, >= 1                 */
    int32_t baro_fuse;        /* substeps per barotropic launch: 0 = library default (7),
                                 1 = one substep per launch pair, 2..8 = that many
                                 substeps per launch on an LDS tile whose halo is as
                                 wide as the substep count (the paper's wide
                                 barotropic halo, Sec. 5.3, applied within one GPU) */
    int32_t salinity;         /* 1: carry salinity S (advected, restored and diffused
                                 like T) and take the buoyancy from the equation of
                                 state eos[] below; 0: temperature only with the
                                 linear b = g alpha (T - t_ref). Ensembles and the
                                 closure network take temperature only.            */
    double dt;                /* baroclinic step (s)                                */
    double chi;               /* AB2 offset: G = (3/2+chi) G^n - (1/2+chi) G^{n-1}  */
    double g;                 /* gravity (m/s^2)                                    */
    double alpha;             /* thermal expansion (1/K): b = g alpha (T - t_ref)   */
    double rho0;              /* reference density (kg/m^3)                         */
    double t_ref;             /* equation-of-state reference temperature (degC)     */
    double kappa;             /* vertical diffusivity = viscosity (m^2/s)           */
    double restore_tau;       /* surface restoring time (s); <= 0 disables          */
    double pgf_weight;        /* eps in [0, 1]: the momentum step takes the hydrostatic
                                 pressure gradient of T^n + eps dt Ghat_T, the tracer
                                 just predicted by AB2 weighted by eps (forward-
                                 backward treatment of internal gravity waves, a
                                 reading of the implicit-explicit AB2 of Sec. 5.2);
                                 the other momentum terms take AB2               */
    double eos[9];            /* with salinity: a0, b0, lambda1, lambda2, mu1, mu2, nu,
                                 t0, s0 of the simplified seawater equation of state
                                 (Roquet et al. 2015 form, the paper's realistic runs
                                 carrying heat and salt, Sec. 6): density anomaly
                                 rho' = -a0 (1 + lambda1 Ta/2 + mu1 z) Ta
                                 + b0 (1 - lambda2 Sa/2 - mu2 z) Sa - nu Ta Sa,
                                 Ta = T - t0, Sa = S - s0, z the depth (m), and
                                 b = -g rho'/rho0; unused without salinity         */
    int32_t momentum_form;    /* 0: flux form (advection of u, v by the face
                                 transports, Coriolis with the spherical metric
                                 term); 1: vector-invariant form, (f + zeta) k x u
                                 + grad(|u|^2/2) + w du/dz with the corner
                                 vorticity reconstructed by WENO upwind of the
                                 transverse velocity (paper Sec. 5.2: WENO
                                 momentum advection on curvilinear grids).
                                 Ensembles take the flux form.                    */
    int32_t reserved2;        /* must be 0                                        */
} ocn_params;

/* Field identifiers. */
typedef enum {
    OCN_FIELD_U = 0,          /* 3D zonal velocity (m/s)                            */
    OCN_FIELD_V = 1,          /* 3D meridional velocity (m/s)                       */
    OCN_FIELD_T = 2,          /* 3D temperature (degC)                              */
    OCN_FIELD_ETA = 3,        /* 2D free surface (m)                                */
    OCN_FIELD_UBT = 4,        /* 2D barotropic transport U (m^2/s)                  */
    OCN_FIELD_VBT = 5,        /* 2D barotropic transport V (m^2/s)                  */
    OCN_FIELD_ETA_MEAN = 6,   /* 2D substep average of eta over the last step       */
    OCN_FIELD_UBT_MEAN = 7,   /* 2D substep average of U over the last step         */
    OCN_FIELD_VBT_MEAN = 8,   /* 2D substep average of V over the last step         */
    OCN_FIELD_W = 9,          /* (nz+1)*ny*nx vertical velocity on z-faces, get only */
    OCN_FIELD_GU_PREV = 10,   /* 3D AB2 history of u (terms other than the pressure
                                 gradient, which is not extrapolated)               */
    OCN_FIELD_GV_PREV = 11,   /* 3D AB2 history of v (likewise)                     */
    OCN_FIELD_GT_PREV = 12,   /* 3D AB2 history of T                                */
    OCN_FIELD_TAUX = 13,      /* 2D zonal wind stress at u-points (N/m^2)           */
    OCN_FIELD_TAUY = 14,      /* 2D meridional wind stress at v-points (N/m^2)      */
    OCN_FIELD_TSTAR = 15,     /* 2D surface restoring temperature (degC)            */
    OCN_FIELD_TREF = 16,      /* nz reference profile of the stored T anomaly        */
    OCN_FIELD_KAPPA = 17,     /* 3D tracer diffusivity on z-faces (m^2/s): slot k is
                                 the face between layers k-1 and k; get returns 0 on
                                 dry faces (and the constant when no closure is
                                 attached); set only with a prescribed-field closure */
    OCN_FIELD_VISC = 18,      /* 3D momentum coefficient on tracer z-faces (m^2/s), get
                                 only: the viscosity of Richardson-number mixing, else
                                 the same as KAPPA; u and v faces take the mean of
                                 their two neighbouring columns */
    OCN_FIELD_U_PRED = 19,    /* 3D AB2-predicted u* (m/s), output of the tendency stage */
    OCN_FIELD_V_PRED = 20,    /* 3D AB2-predicted v* (m/s)                           */
    OCN_FIELD_T_PRED = 21,    /* 3D AB2-predicted T* (degC)                          */
    OCN_FIELD_GU_SLOW = 22,   /* 2D barotropic slow forcing: depth integral of the
                                 AB2 u tendency (m^2/s^2), output of the tendency stage */
    OCN_FIELD_GV_SLOW = 23,   /* 2D the same for v                                   */
    OCN_FIELD_S = 24,         /* 3D salinity (g/kg), with salinity only; as for T the
                                 first set fixes the per-level reference profile   */
    OCN_FIELD_GS_PREV = 25,   /* 3D AB2 history of S                                */
    OCN_FIELD_SSTAR = 26,     /* 2D surface restoring salinity (g/kg)               */
    OCN_FIELD_S_PRED = 27,    /* 3D AB2-predicted S*                                 */
    OCN_FIELD_SREF = 28       /* nz reference profile of the stored S anomaly         */
} ocn_field;

/* Stages of one step, in the order ocn_step runs them (paper Sec. 5.1-5.3;
 * the order is a reading of the time-stepping sequence, whose figure the
 * paper's text lacks):
 *  MIXING      the face diffusivity diagnosed from the current state
 *              (convective adjustment, Richardson-number mixing or the
 *              network of an attached closure; nothing otherwise);
 *  TENDENCY    w and hydrostatic pressure, the tendencies, the AB2 predictor
 *              (U_PRED, V_PRED, T_PRED, new histories) and the slow forcing
 *              (GU_SLOW, GV_SLOW);
 *  BAROTROPIC  the substeps from ETA, UBT, VBT and the slow forcing (new ETA,
 *              UBT, VBT and the window averages);
 *  COLUMN      backward-Euler vertical diffusion of the predicted fields and
 *              the depth-mean correction with UBT_MEAN, VBT_MEAN (new U, V, T). */
typedef enum {
    OCN_STAGE_MIXING = 0,
    OCN_STAGE_TENDENCY = 1,
    OCN_STAGE_BAROTROPIC = 2,
    OCN_STAGE_COLUMN = 3
} ocn_stage;

typedef struct ocn_diag {
    int64_t step;             /* steps taken                                        */
    double time;              /* model time (s)                                     */
    double tracer_content;    /* sum V_c T over wet cells (degC m^3)                */
    double volume;            /* sum A_c eta over wet columns (m^3)                 */
    double volume_mean;       /* sum A_c eta_mean over wet columns (m^3)            */
    double kinetic_energy;    /* 1/2 sum (V_u u^2 + V_v v^2) (m^5/s^2)              */
    double max_abs_u, max_abs_v, max_abs_w;
    double t_min, t_max;      /* over wet cells                                     */
    double eta_min, eta_max;  /* over wet columns                                   */
    double cfl_adv;           /* max(|u| dt/dx, |v| dt/dy, |w| dt/dz)               */
    double wet_area;          /* sum A_c over wet columns (m^2)                     */
    int64_t nonfinite;        /* cells with a non-finite u, v, T (or S), plus columns with
                                 a non-finite eta, U or V                           */
    double cfl_bt;            /* barotropic CFL of a substep: max over wet columns of
                                 sqrt(g H) (dt / n_substeps) sqrt(1/dx^2 + 1/dy^2)   */
    double salt_content;      /* sum V_c S over wet cells (g/kg m^3; 0 without salinity) */
} ocn_diag;

typedef struct ocn_grid ocn_grid;
typedef struct ocn_state ocn_state;

/* Version of this ABI (OCN_ABI_VERSION). */
uint32_t ocn_abi_version(void);

/* Text of the last error on the calling thread; valid until its next call. */
const char* ocn_last_error(void);

/* Build the grid: copies desc, dz and kbottom (the caller may free them after
 * the call) and derives metrics and masks on the host. Finite-volume C-grid of
 * paper Sec. 5.2 on a Cartesian beta-plane or a lat-lon sphere (Sec. 6). */
int  ocn_grid_create(const ocn_grid_desc* desc, ocn_grid** out);
void ocn_grid_destroy(ocn_grid* grid);

/* Device bytes one state of this grid and precision needs. */
int ocn_state_arena_bytes(const ocn_grid* grid, const ocn_params* params, size_t* bytes);

/* Create a state at rest (u = v = T = eta = U = V = 0, no forcing) inside the
 * caller's device arena (256-byte aligned, at least ocn_state_arena_bytes bytes)
 * on the caller's HIP stream (hipStream_t, NULL for the default stream). The
 * grid must outlive the state. The arena is written only by this library until
 * ocn_state_destroy. */
int  ocn_state_init(const ocn_grid* grid, const ocn_params* params, void* device_arena,
                    size_t arena_bytes, void* hip_stream, ocn_state** out);
void ocn_state_destroy(ocn_state* state);

/* Copy a host field in (set) or out (get); count must equal the field's size.
 * Set stores u and v with dry points zeroed. Setting TREF is allowed only
 * before T is first set; otherwise the first set of T takes as reference the
 * mean of that T over the wet cells of each level. Both calls synchronise the
 * stream. */
int ocn_set_field(ocn_state* state, int32_t field, const double* host, size_t count);
int ocn_get_field(ocn_state* state, int32_t field, double* host, size_t count);

/* AB2 start flag: 1 makes the next step forward Euler (paper Sec. 5.2 AB2).
 * A new state starts with it set. Setting fields leaves it as it is, so that
 * a caller can restore a state together with its AB2 histories; a caller
 * that replaces u, v or T without their histories sets it to 1. */
int ocn_set_first_step(ocn_state* state, int32_t first);
int ocn_get_first_step(ocn_state* state, int32_t* first);

/* Enqueue n >= 0 steps on the state's stream; returns without waiting. Each
 * step: fused tendency + AB2 kernel (w and hydrostatic pressure integrated in
 * the vertical march, slow barotropic forcing summed in FP64), the barotropic
 * substeps (FP64, forward-backward), then the column kernel (backward-Euler
 * vertical diffusion of T, u, v and the depth-mean correction of u, v). */
int ocn_step(ocn_state* state, int32_t n);

/* Reduce diagnostics on the device (compensated FP64 sums in a fixed order),
 * synchronise and copy them out. Returns OCN_E_UNSTABLE (with *out filled)
 * when any prognostic value is non-finite. */
int ocn_diagnostics(ocn_state* state, ocn_diag* out);

/* The same diagnostics for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * per-workgroup partial sums and the reduced values live in a fixed device
 * array of the library instead of the state's arena, and the call allocates
 * nothing. The array holds the partials of grids of up to 8,388,608 columns
 * (nx ny; larger grids return OCN_E_UNSUPPORTED) and is shared by every call
 * on a GPU: calls that overlap on one GPU (several streams or host threads)
 * race and must be serialised by the caller. Results equal ocn_diagnostics'.
 * Synchronises the stream. */
int ocn_diagnostics_noalloc(ocn_state* state, ocn_diag* out);

/* Wait for all work enqueued on the state's stream. */
int ocn_synchronize(ocn_state* state);

/* Enqueue one stage of a step (ocn_stage) and nothing else: no step count,
 * time or AB2 start flag changes (the flag is read by the TENDENCY stage).
 * Running MIXING, TENDENCY, BAROTROPIC and COLUMN in turn enqueues the same
 * kernels as one ocn_step. For stage-by-stage checks: set a stage's inputs
 * (ocn_set_field), run it, read its outputs. OCN_E_INVALID for an unknown
 * stage. Asynchronous. */
int ocn_debug_run_stage(ocn_state* state, int32_t stage);

/* Batched ensembles (many independent basins stepped together). An ensemble
 * holds n member states of possibly different grids but one ocn_params, laid
 * out in one caller arena of ocn_ensemble_arena_bytes. ocn_ensemble_step
 * advances every member with one launch of the tendency kernel and one of the
 * column kernel for the whole ensemble, and one barotropic launch per group of
 * fused substeps; after the first step (forward Euler) the launches of a step
 * are captured once into a HIP graph on the ensemble's stream and replayed
 * (no capture when the stream is NULL). Each member's arithmetic is the same
 * as when it is stepped alone with the same tile settings, so results are
 * bitwise identical to stepping the members one by one. Motivation: climate
 * uncertainty needs ensembles of simulations (paper Sec. 3).
 *
 * ocn_ensemble_member returns a borrowed handle of member m for the state
 * calls (set/get fields, diagnostics, checkpoints); do not destroy it.
 * ocn_ensemble_set_tiles selects the tendency workgroup rows (4 or 8; 0 =
 * precision default), the barotropic substeps per launch (2..8; 0 = 7, the
 * default) and the schedule: persistent = 0 launches one workgroup per tile
 * table entry; persistent = 1 launches, per stage, as many workgroups as fit
 * on the device at once, which take the entries from eight per-XCD atomic
 * counters in the ensemble's arena (zeroed by a kernel at the start of each
 * step) and leave when all are taken. Every choice gives bitwise-identical
 * results. ocn_ensemble_autotune times trial_steps steps of each choice
 * (rows x substeps x schedule), keeps the fastest, restores the state it
 * started from and reports the choice and its time per step; any output
 * pointer may be NULL. */
typedef struct ocn_ensemble ocn_ensemble;
int  ocn_ensemble_arena_bytes(const ocn_grid* const* grids, int32_t n, const ocn_params* params, size_t* bytes);
int  ocn_ensemble_init(const ocn_grid* const* grids, int32_t n, const ocn_params* params, void* device_arena,
                       size_t arena_bytes, void* hip_stream, ocn_ensemble** out);
void ocn_ensemble_destroy(ocn_ensemble* ens);
int  ocn_ensemble_member(ocn_ensemble* ens, int32_t m, ocn_state** member);
int  ocn_ensemble_step(ocn_ensemble* ens, int32_t n);
int  ocn_ensemble_set_tiles(ocn_ensemble* ens, int32_t tend_rows, int32_t baro_fuse, int32_t persistent);
int  ocn_ensemble_autotune(ocn_ensemble* ens, int32_t trial_steps, int32_t* tend_rows, int32_t* baro_fuse,
                           int32_t* persistent, double* ms_per_step);

/* Per-column closure network: Linear -> ReLU -> Linear -> ReLU -> Linear with
 * BF16 operands on the matrix cores and FP32 accumulation, FP32 master weights
 * and Adam; it maps a column's features to its vertical-diffusivity profile
 * (paper Sec. 3 motivates learned parameterizations, Sec. 6 uses a
 * vertical-mixing closure). Parameters
 * are packed FP32: W1 (din x h1, row-major), b1, W2 (h1 x h2), b2, W3
 * (h2 x dout), b3. Batches are device pointers to FP32 row-major matrices,
 * rows <= max_batch: x (rows x din), targets and outputs (rows x dout).
 * ocn_mlp_gradients returns the mean-squared loss sum (y - t)^2 / (2 rows dout)
 * and its gradients (synchronises); ocn_mlp_train_step also applies one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr, and when
 * loss is non-NULL synchronises to return the loss before the update.
 * ocn_mlp_set_params resets the Adam moments. Inference (ocn_mlp_forward and
 * the closure) runs all three layers in one kernel with the weights held in
 * LDS when din % 8 == 0, din <= 256, h1 and h2 are multiples of 32 up to 128
 * and dout <= 128; other shapes run layer by layer. Both round the same
 * operands to BF16; they differ only in FP32 accumulation order. */
typedef struct ocn_mlp ocn_mlp;
int  ocn_mlp_arena_bytes(int32_t din, int32_t h1, int32_t h2, int32_t dout, int32_t max_batch, size_t* bytes);
int  ocn_mlp_init(int32_t din, int32_t h1, int32_t h2, int32_t dout, int32_t max_batch, void* device_arena,
                  size_t arena_bytes, void* hip_stream, ocn_mlp** out);
void ocn_mlp_destroy(ocn_mlp* net);
int  ocn_mlp_param_count(const ocn_mlp* net, size_t* count);
int  ocn_mlp_set_params(ocn_mlp* net, const float* host, size_t count);
int  ocn_mlp_get_params(ocn_mlp* net, float* host, size_t count);
int  ocn_mlp_forward(ocn_mlp* net, const float* x_dev, int32_t rows, float* y_dev);
int  ocn_mlp_gradients(ocn_mlp* net, const float* x_dev, const float* t_dev, int32_t rows, float* grads_host,
                       size_t count, float* loss_host);
int  ocn_mlp_train_step(ocn_mlp* net, const float* x_dev, const float* t_dev, int32_t rows, float lr,
                        float* loss_host);

/* Vertical-diffusivity closure (paper Sec. 5.2 implicit vertical diffusion;
 * Sec. 3 motivates learned parameterizations, Sec. 6 runs with a
 * vertical-mixing closure). With a closure attached the implicit diffusion
 * uses a diffusivity per z-face and column: T on its own faces, u and v the
 * mean of their two neighbouring columns' faces. Two modes:
 *  - net == NULL: a prescribed field, set with ocn_set_field(OCN_FIELD_KAPPA)
 *    (initialised to the constant kappa) or ocn_closure_kappa;
 *  - net != NULL: at the start of every ocn_step the state's columns are fed
 *    to the network (features as ocn_closure_features, normalised by norm:
 *    din means then din standard deviations, host FP32) and its outputs mapped
 *    as ocn_closure_kappa does; the network needs din >= 4 nz + 3 and
 *    dout == nz, and its current weights are read at every step.
 * The workspace (device, 256-byte aligned, ocn_closure_workspace_bytes) holds
 * the face field and, with a network, its activations for every column; it
 * must outlive the attachment. The network must outlive it too. Any nz the
 * state takes (<= 128) is supported. Ensembles and checkpoints do not carry a
 * closure. */
int ocn_closure_workspace_bytes(const ocn_state* state, const ocn_mlp* net, size_t* bytes);
int ocn_closure_attach(ocn_state* state, const ocn_mlp* net, const float* norm, size_t norm_count,
                       void* device_workspace, size_t workspace_bytes);
int ocn_closure_detach(ocn_state* state);
/* Convective adjustment in the prescribed-field mode (paper Sec. 5.1: the
 * diffusivity is a diagnostic of the current state; Sec. 6 runs a
 * vertical-mixing closure): with kappa_conv > 0 every step starts by setting
 * the face field to kappa_conv on interior wet faces where N^2 = g alpha dT/dz
 * < 0 (denser water above) and to the constant kappa elsewhere; kappa_conv <= 0
 * turns it off (the field keeps its last values). Needs a closure attached
 * with net == NULL (else OCN_E_STATE); synchronises the stream. */
int ocn_closure_convective(ocn_state* state, double kappa_conv);
/* Richardson-number vertical mixing in the prescribed-field mode (paper Sec. 6
 * runs a Richardson-number-based parameterization of shear and convective
 * mixing and gives no formula; this is the Pacanowski-Philander form). With
 * nu0 > 0 every step starts by diagnosing, on each interior wet z-face from
 * the current state, N^2 = g alpha dT/dz and S^2 = |d(u_c, v_c)/dz|^2 (u, v
 * averaged to the cell centre); where N^2 < 0 the viscosity and diffusivity
 * are conv, else with Ri = N^2 / max(S^2, 1e-16) and r = 1 / (1 + alpha Ri):
 * viscosity nu = nu0 r^2 + nu_b (u and v), diffusivity nu r + kappa_b (T).
 * The faces of the current state are diagnosed at once (OCN_FIELD_KAPPA,
 * OCN_FIELD_VISC). nu0 <= 0 turns it off and sets every face back to the
 * constant kappa; enabling it turns convective adjustment off and enabling
 * that turns it off. Needs a closure attached with net == NULL (else
 * OCN_E_STATE); alpha, nu_b, kappa_b, conv must be finite and >= 0;
 * synchronises the stream. */
int ocn_closure_richardson(ocn_state* state, double nu0, double alpha, double nu_b, double kappa_b,
                           double conv);
/* Network inputs of every column of the current state into x (device FP32,
 * (ny nx) x din row-major, row j nx + i), din >= 4 nz + 3 and 64 (din + 1) 4
 * bytes <= 64 KiB. Order: T (nz levels, bottom first), u and v averaged to
 * the centre (nz each), N^2 = g alpha dT/dz on face k (nz; face 0 and dry
 * faces 0), wind stress averaged to the centre (2), surface restoring flux
 * dz_top (T* - T_top) / tau in K m/s (1, 0 when off), zeros. Wet entries are
 * (x - mean) / std with norm_dev (device FP32, din means then din deviations)
 * or raw when norm_dev is NULL; dry entries are 0. Asynchronous. */
int ocn_closure_features(ocn_state* state, int32_t din, const float* norm_dev, float* x_dev);
/* Network outputs (device FP32, (ny nx) rows of leading dimension ldy >= nz:
 * slot k = log10 diffusivity on z-face k, between layers k-1 and k; slot 0 is
 * unused) to the attached face field: a wet interior face takes 10^y clipped
 * to [1e-7, 1] m^2/s, or the constant kappa where y is not finite; dry faces
 * take 0. Asynchronous. */
int ocn_closure_kappa(ocn_state* state, const float* y_dev, int32_t ldy);

/* Checkpoint and resume. ocn_checkpoint_bytes reports the size of a
 * checkpoint; ocn_checkpoint_save copies the state as stored on the device
 * (prognostic fields including halos, AB2 history, barotropic state and
 * averages, the reference profile, step count, time and the AB2 start flag)
 * into the caller's host buffer; ocn_checkpoint_load restores it into a state
 * of the same grid, precision and halo. Forcing fields are not included: set
 * them again. Stepping on from a loaded checkpoint is bitwise identical to
 * stepping on from the saved state. Both calls synchronise the stream;
 * a size or grid mismatch returns OCN_E_INVALID. */
int ocn_checkpoint_bytes(ocn_state* state, size_t* bytes);
int ocn_checkpoint_save(ocn_state* state, void* host, size_t bytes);
int ocn_checkpoint_load(ocn_state* state, const void* host, size_t bytes);

/* The same steps through a HIP graph: the first call that steps past the
 * forward-Euler start captures the kernels of one step (thread-local capture
 * on the state's stream) and every later step replays that graph, which
 * removes the per-launch host cost on small grids. The start step and steps
 * taken while stage timing is on run eagerly. The graph is rebuilt after a
 * closure is attached or detached. The state's stream must not be the null
 * stream (OCN_E_UNSUPPORTED). Results are bitwise those of ocn_step. */
int ocn_step_graph(ocn_state* state, int32_t n);

/* Per-stage timing with HIP events recorded on the state's stream. While
 * enabled (enable = 1), every ocn_step records an event at its start, after
 * the closure update, after the tendency kernel, after the barotropic
 * substeps and after the column kernel. ocn_stage_times synchronises the
 * stream, writes up to n accumulated stage times in milliseconds (0 tendency,
 * 1 barotropic substeps, 2 column solve and correction, 3 closure update) and
 * the number of timed steps, then clears the accumulators. Enabling or
 * disabling also clears them. */
int ocn_stage_timing(ocn_state* state, int32_t enable);
int ocn_stage_times(ocn_state* state, double* ms, int32_t n, int64_t* steps);

#ifdef __cplusplus
}
#endif
#endif
