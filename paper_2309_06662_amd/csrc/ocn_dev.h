// ocn_dev.h -- device-side view of one ocean state, shared by the HIP kernels
// and the host runtime of the library.
//
// Layout in HBM. Every 3D field is x-fastest [k][j][i] with a halo of h cells
// on each side in x and y and none in z. Rows are padded so that the interior
// of every row starts on a 128-byte boundary; the pointers below point at the
// interior origin (i = 0, j = 0, k = 0), so (i, j) run from -h to n + h - 1.
// 2D fields (FP64 barotropic state, column sums, forcing) use the same
// horizontal padding with their own pitch; the int32 wet-layer counts carry one
// more halo cell than the fields, for the masks at the far end of a stencil.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct ocn_mlp;

namespace ocn {

// Diagnostics slots reduced on the device.
enum DiagSlot {
    DG_TRACER = 0, DG_VOLUME, DG_VOLUME_MEAN, DG_KE, DG_WET_AREA, DG_SALT,  // compensated sums
    DG_NSUM = 6,
    DG_MAX_U = 6, DG_MAX_V, DG_MAX_W, DG_CFL, DG_T_MAX, DG_NEG_T_MIN, DG_ETA_MAX, DG_NEG_ETA_MIN,  // maxima
    DG_NONFINITE = 14,
    DG_COUNT = 15
};

struct DevState {
    // sizes
    int nx, ny, nz, h;
    int hk;            // halo of the wet-layer counts: h + 1 (velocity masks at stencil ends)
    int periodic_x, periodic_y, latlon;
    int p3;            // row pitch of 3D fields (elements of the field type)
    int p2;            // row pitch of 2D double fields
    int ox2;           // offset of the interior in a 2D row (elements)
    int pk;            // row pitch of the int32 wet-layer counts
    long long plane3;  // (ny + 2h) * p3
    // 3D fields of the field type (double or float), interior origin
    void *u, *v, *t;        // state; t holds T - tref(k)
    void *us, *vs, *ts;     // AB2 predictor phi*
    void *gu, *gv;          // AB2 history G^{n-1} of u, v (other terms than the
                            // pressure gradient), overwritten with G^n
    void *gt, *gt_out;      // AB2 history of T: G^{n-1} is read from gt and G^n
                            // written to gt_out (the host swaps them every step)
    // salinity (when salinity != 0): S - sref(k), its predictor, and its
    // double-buffered AB2 history like T's
    int salinity;
    int vi;           // momentum advection: 0 flux form, 1 vector-invariant form
    void *s, *ss, *gs, *gs_out;
    // 2D FP64
    double *eta, *ubt, *vbt;             // barotropic state
    double *se, *su, *sv;                // window sums of eta^q; transport sums of U^l, V^l
    double *eta_mean, *ubt_mean, *vbt_mean;
    double *gU, *gV;                     // slow forcing: depth integral of the AB2 momentum tendency
    double *hu, *hv;                     // depth of u and v columns
    double *cumh;                        // nz + 1: depth of a column of K wet layers, K = 0..nz
                                         // (summed as hu, hv are: the same doubles)
    double *cu, *cv;                     // sum_k dz u m_u of the current u, v (vertical-transport seed)
    double *taux, *tauy;                 // wind stress
    double *tstar;                       // restoring target minus tref(top)
    double *sstar;                       // salinity restoring target minus sref(top) (salinity only)
    double *scratch2d;                   // one 2D field of scratch
    double *eta2, *ubt2, *vbt2;          // second buffers of the temporally blocked substeps
    double *sfu, *sfv;                   // window sums of U^q, V^q
    double *baro_a;                      // M + 1 substep weights a_q (a_0 unused)
    double *baro_A;                      // M tail sums A_l = sum_{q>l} a_q
    int baro_m;                          // substeps per step: Ns + Ns/2
    // int32 wet layers per column counted from the surface, with a halo of hk
    // (periodic images wrapped, zero beyond walls)
    int* kb;
    // row metrics, index j from -h to ny + h (FP64), interior origin
    double *dxc, *dxv, *area, *fcor, *metric;
    double *fcor_s;   // Coriolis parameter on the south face of each row (vector-invariant form)
    double dy;
    // level tables
    double* dz;       // nz
    double* dzc;      // nz + 1: centre spacing below layer k (dzc[0] and dzc[nz] unused)
    double* tref;     // nz
    void* dtr;        // nz * 4 of the field type: tref(k+o) - tref(k), o = -2, -1, +1, +2
    // salinity only: the reference profile of S and its steps (as tref, dtr);
    // the buoyancy of anomalies b' = T'(eT + qT T' + qTS S') + S'(eS + qS S')
    // with eT, eS per level (2 nz of the field type) and, for N^2 at any depth
    // in FP64, the equation-of-state constants and layer-centre depths
    double* sref;
    void* dsr;
    void* eos_tab;
    double eos_qT, eos_qTS, eos_qS;
    double eos[9];    // a0, b0, lambda1, lambda2, mu1, mu2, nu, t0, s0
    double* zc;       // nz depths of the layer centres (m, positive down)
    // constant-diffusivity solve, eliminated from the surface down: per level k
    // of the field type {1 / b'_k, c_k / b'_{k+1}, 1 / b''_k, a_k}, with b' the
    // pivot of a layer above the bottom, b'' the pivot of layer k when it is
    // the bottom layer, a_k = -dt kappa / dzc_k and c_k = a_{k+1} (0 at the top)
    void* thomas_tab; // 4 nz
    // vertical diffusivity on z-faces (3D of the field type, slot k = face
    // between layers k-1 and k, with periodic images), or null for the constant
    void* kw;
    void* kv;       // viscosity on z-faces for u and v (Richardson mixing), or null: they use kw
    // diagnostics scratch
    double* diag_part;  // blocks * DG_COUNT
    double* diag_out;   // DG_COUNT
    int diag_blocks;
    // scalars
    double dt, chi, g, alpha, rho0, kappa, restore_inv;
    double pgf_w;   // eps: the momentum step's pressure is that of T^n + eps dt Ghat_T
    int n_substeps;
    int baro_fuse;  // substeps per barotropic launch
    int tend_ty;    // rows of threads per tendency workgroup (4 or 8; 0 = precision default)
};

template <typename R>
__device__ __forceinline__ R* f3(void* p) { return static_cast<R*>(p); }

__host__ __device__ inline long long idx3(const DevState& s, int i, int j, int k) {
    return (long long)k * s.plane3 + (long long)j * s.p3 + i;
}
__host__ __device__ inline long long idx2(const DevState& s, int i, int j) {
    return (long long)j * s.p2 + i;
}
__host__ __device__ inline long long idxk(const DevState& s, int i, int j) {
    return (long long)j * s.pk + i;
}

// Visit every periodic image (x, y) of interior point (i, j) that lies inside
// the halo band of width ext (ext_x, ext_y), excluding (i, j) itself.
template <class F>
__device__ __forceinline__ void for_each_image(const DevState& s, int i, int j, int ext, F&& f) {
    int xlo = i, xhi = i, ylo = j, yhi = j;
    if (s.periodic_x) {
        while (xlo - s.nx >= -ext) xlo -= s.nx;
        while (xhi + s.nx < s.nx + ext) xhi += s.nx;
    }
    if (s.periodic_y) {
        while (ylo - s.ny >= -ext) ylo -= s.ny;
        while (yhi + s.ny < s.ny + ext) yhi += s.ny;
    }
    for (int y = ylo; y <= yhi; y += s.ny)
        for (int x = xlo; x <= xhi; x += s.nx)
            if (x != i || y != j) f(x, y);
}

// The periodic images of column (i, j) within a halo band of width ext, as
// element offsets in a 3D field (the same on every level), computed without
// a capturing lambda so they stay in registers: at most one image per
// periodic direction plus the corner. n > 3 (a domain narrower than twice the
// band) tells the caller to fall back to for_each_image.
struct Images {
    int n;
    long long o0, o1, o2;
};
__device__ __forceinline__ Images column_images(const DevState& s, int i, int j, int ext) {
    Images im{0, 0, 0, 0};
    if ((s.periodic_x && s.nx < 2 * ext) || (s.periodic_y && s.ny < 2 * ext)) {
        im.n = 4;
        return im;
    }
    long long ox = 0, oy = 0;
    if (s.periodic_x) ox = (i < ext) ? s.nx : ((i >= s.nx - ext) ? -s.nx : 0);
    if (s.periodic_y) oy = (j < ext) ? (long long)s.ny * s.p3 : ((j >= s.ny - ext) ? -(long long)s.ny * s.p3 : 0);
    if (ox != 0) im.o0 = ox, im.n = 1;
    if (oy != 0) {
        if (im.n == 0) im.o0 = oy, im.n = 1;
        else im.o1 = oy, im.o2 = ox + oy, im.n = 3;
    }
    return im;
}

// Launchers (defined in the kernel translation units).
template <typename R> hipError_t launch_tendency(const DevState& s, int first, hipStream_t st);
template <typename R> hipError_t launch_column(const DevState& s, hipStream_t st);
template <typename R> hipError_t launch_colsum(const DevState& s, hipStream_t st);
// closure inputs/outputs (k_closure.hip)
size_t features_lds(int din);
template <typename R> hipError_t launch_fill(void* p, long long n, double v, hipStream_t st);
template <typename R>
hipError_t launch_convective(const DevState& s, double kappa_conv, double kappa0, hipStream_t st);
// Richardson-number mixing constants (Pacanowski-Philander form)
struct RiParams {
    double nu0, alpha, nu_b, kappa_b, conv;
};
template <typename R> hipError_t launch_richardson(const DevState& s, const RiParams& p, hipStream_t st);
template <typename R>
hipError_t launch_features(const DevState& s, int din, const float* norm, void* out, int out_bf16, hipStream_t st);
template <typename R>
hipError_t launch_kappa_map(const DevState& s, const float* Y, int ldy, double kappa0, hipStream_t st);
// closure network inference (k_mlp.hip): BF16 X (rows x din) -> FP32 Y (rows x dout)
void mlp_shape(const ::ocn_mlp* net, int* din, int* h1, int* h2, int* dout);
hipError_t mlp_infer(const ::ocn_mlp* net, const uint16_t* Xb, int rows, uint16_t* H1b, uint16_t* H2b, float* Y,
                     hipStream_t st);
template <typename R> hipError_t launch_diagnostics(const DevState& s, hipStream_t st);
// the fixed diagnostics scratch of a device (k_diag.hip): its address and capacity in workgroups
hipError_t diag_scratch(int device, double** ptr, int* max_blocks);
template <typename R> hipError_t launch_w_faces(const DevState& s, double* out_faces_dev, hipStream_t st);
hipError_t launch_barotropic(const DevState& s, hipStream_t st);
int tend_tile_rows(int precision_bytes, int ty_choice);

// Batched launches over an ensemble: members is a device array of states,
// tiles a device table of (member, tile x, tile y[, field]) entries. With a
// queue (8 zeroed counters per launch, device memory) the launch is instead a
// grid of persistent workgroups, as many as fit on the device at once, that
// take table entries from per-XCD atomic counters until all are done (see
// for_each_queued_tile); without one, one workgroup per entry.
template <typename R>
hipError_t launch_tendency_batched(const DevState* members, const int4* tiles, int ntiles, int ty, int first,
                                   int* queue, hipStream_t st);
template <typename R>
hipError_t launch_column_batched(const DevState* members, const int4* tiles, int ntiles, int max_nz, int* queue,
                                 hipStream_t st);
int baro_substeps(int n_substeps);  // Ns + Ns/2
// queue: 8 counters per substep-group launch, baro_launches(...) groups
hipError_t launch_barotropic_batched(const DevState* members, int n_members, const int4* tiles, int ntiles,
                                     int n_substeps, int fuse, double dt, int* queue, hipStream_t st);
int baro_launches(int n_substeps, int fuse);
// zero n counters (a kernel, so that it can sit in a captured graph)
hipError_t launch_zero_counters(int* p, int n, hipStream_t st);
// workgroups of a kernel that fit on the current device at once
int resident_workgroups(const void* kernel, int block_threads);
// Hardware workgroups are dealt to the 8 XCDs round-robin; give XCD x the
// contiguous range of tiles [x*q + min(x, r), ...) of a tile order, so that
// neighbouring tiles share an L2 and read each other's halos from it.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int x = b % 8, slot = b / 8;
    return (x < r) ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// Persistent workgroups over a tile table of n entries, dealt to the 8 XCDs
// round-robin: a workgroup on XCD x (= blockIdx.x mod 8) takes the entries
// x, x+8, x+16, ... (the entries the hardware would have given that XCD, so
// neighbouring tiles still share an L2) by atomic increments of counter x,
// then helps the other XCDs' counters in turn. No workgroup waits for
// another: each leaves once all eight counters have passed their ends, so
// the grid drains whatever its size. f(entry) runs with the whole workgroup.
template <typename F>
__device__ __forceinline__ void for_each_queued_tile(int* q, const int n, F&& f) {
    __shared__ int s_slot;
    const int x = blockIdx.x & 7;
    const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
    for (int d = 0; d < 8; ++d) {
        const int qx = (x + d) & 7;
        const int nq = (n - qx + 7) / 8;  // entries qx, qx+8, ... below n
        for (;;) {
            __syncthreads();  // the previous entry is done with LDS and s_slot
            if (lead) s_slot = atomicAdd(&q[qx], 1);
            __syncthreads();
            const int slot = s_slot;
            if (slot >= nq) break;
            f(qx + 8 * slot);
        }
    }
}

// Most levels a state may have (the column solve's register buckets and the
// tendency kernel's per-level LDS table are sized for it).
constexpr int kMaxLevels = 128;
constexpr int kBaroTileX = 64, kBaroTileY = 24;
// substeps per barotropic launch unless chosen: 7 keeps the 64 x 24 tile's LDS
// (77 KB) and registers (128) within two workgroups per CU
constexpr int kBaroFuseDefault = 7;

}  // namespace ocn
