// ocn_api.hip -- host runtime behind the C ABI declared in include/ocn.h.
//
// Builds the grid metrics and masks on the host, lays the state out in the
// caller's device arena, moves fields between host doubles and the padded
// device layout, and enqueues the kernels of a step on the caller's stream.
#include "ocn.h"
#include "ocn_dev.h"

#include <algorithm>
#include <utility>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using ocn::DevState;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(OCN_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr double kPi = 3.14159265358979323846;

}  // namespace

namespace ocn {
int set_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace ocn

struct ocn_grid {
    ocn_grid_desc d;
    int nx, ny, nz, h;
    std::vector<double> dz, dzc;
    std::vector<int32_t> kb;              // ny * nx interior
    // row metrics for j = -h .. ny + h (index j + h)
    std::vector<double> dxc, dxv, area, fcor, metric, fcor_s;
    double dy;
    int row(int j) const { return j + h; }
};

struct ocn_state {
    const ocn_grid* g = nullptr;
    ocn_params p{};
    DevState d{};
    hipStream_t st = nullptr;
    void* arena = nullptr;
    size_t bytes = 0;
    int esize = 8;          // bytes per element of the 3D field type
    int first = 1;
    int64_t step = 0;
    double time = 0.0;
    bool t_set = false;
    std::vector<double> tref;   // nz
    std::vector<double> tstar;  // ny * nx, absolute
    bool s_set = false;         // salinity: reference profile fixed by the first set of S
    std::vector<double> sref;   // nz (salinity)
    std::vector<double> sstar;  // ny * nx, absolute (salinity)
    // stage timing (events recorded on the state's stream)
    bool timing = false;
    std::vector<hipEvent_t> events;  // 4 per timed step
    int64_t timed_steps = 0;
    // host-side layout facts
    size_t ox3 = 0, ox2 = 0, oxk = 0;
    size_t n3 = 0, n2 = 0, nk = 0;  // padded element counts
    // vertical-diffusivity closure (null net: prescribed field)
    bool closure = false;
    const ocn_mlp* net = nullptr;
    int din = 0, h1 = 0, h2 = 0, dout = 0;
    float* norm = nullptr;        // device: mean[din], std[din]
    uint16_t *xb = nullptr, *h1b = nullptr, *h2b = nullptr;
    float* y = nullptr;
    double kappa_conv = 0.0;      // > 0: convective adjustment into the prescribed field
    bool ri_on = false;           // Richardson-number mixing into the prescribed field
    ocn::RiParams ri{};
    void* kv_ws = nullptr;        // the workspace's viscosity field (interior origin)
    // the two tracer-history buffers; d.gt is the one the next step reads
    void* gtb[2] = {nullptr, nullptr};
    void swap_history() {  // G^n becomes the history the next step reads
        std::swap(d.gt, d.gt_out);
        std::swap(d.gs, d.gs_out);
    }
    double cfl_bt = 0.0;  // barotropic CFL of a substep (static: grid and parameters)
    // one step captured as a HIP graph per history buffer (ocn_step_graph)
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int parity() const { return d.gt == gtb[0] ? 0 : 1; }
};

namespace {

void drop_graph(ocn_state* s) {
    for (int q = 0; q < 2; ++q) {
        if (s->exec[q]) (void)hipGraphExecDestroy(s->exec[q]);
        if (s->graph[q]) (void)hipGraphDestroy(s->graph[q]);
        s->exec[q] = nullptr;
        s->graph[q] = nullptr;
    }
}

int record(ocn_state* s) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    s->events.push_back(e);
    HIPCHK(hipEventRecord(e, s->st));
    return OCN_OK;
}

void drop_events(ocn_state* s) {
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    s->events.clear();
    s->timed_steps = 0;
}

}  // namespace

namespace {

// Wrap an index into the interior for periodic directions; -1 outside a wall.
int wrap(int i, int n, bool periodic) {
    if (i >= 0 && i < n) return i;
    if (!periodic) return -1;
    int r = i % n;
    return r < 0 ? r + n : r;
}

struct Layout {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t off = round_up(total, 256);
        total = off + round_up(bytes, 256);
        return off;
    }
};

// Offsets of every array of a state in the arena (same order as assign()).
struct Plan {
    size_t esize, a3, ox3, p3, rows, n3;
    size_t ox2, p2, n2;
    size_t oxk, pk, nk;
    size_t nrow;  // metric rows
    size_t diag_blocks;
    int nf3, nf2;  // 3D and 2D arrays of the state (more with salinity)
    size_t off_f3[14], off_f2[25], off_bw, off_kb, off_rows[6], off_dz, off_dzc, off_tref, off_dtr, off_tab, off_cumh;
    size_t off_sref, off_dsr, off_eos, off_zc;
    size_t off_part, off_out;
    size_t total;
};

Plan make_plan(const ocn_grid* g, int precision, int n_substeps, int salinity) {
    Plan P{};
    P.nf3 = salinity ? 14 : 10;
    P.nf2 = salinity ? 25 : 24;
    P.esize = precision == OCN_FP32 ? 4 : 8;
    const size_t h = g->h;
    P.rows = g->ny + 2 * h;
    const size_t a3 = 128 / P.esize;
    P.ox3 = round_up(h, a3);
    P.p3 = round_up(P.ox3 + g->nx + h, a3);
    P.n3 = P.p3 * P.rows * g->nz;
    P.ox2 = round_up(h, 16);
    P.p2 = round_up(P.ox2 + g->nx + h, 16);
    P.n2 = P.p2 * P.rows;
    P.oxk = round_up(h + 1, 32);
    P.pk = round_up(P.oxk + g->nx + h + 1, 32);
    P.nk = P.pk * (g->ny + 2 * (h + 1));
    P.nrow = g->ny + 2 * h + 1;
    P.diag_blocks = ((g->nx + 63) / 64) * ((g->ny + 3) / 4);
    Layout L;
    for (int q = 0; q < P.nf3; ++q) P.off_f3[q] = L.add(P.n3 * P.esize);
    for (int q = 0; q < P.nf2; ++q) P.off_f2[q] = L.add(P.n2 * sizeof(double));
    P.off_kb = L.add(P.nk * sizeof(int32_t));
    for (auto& o : P.off_rows) o = L.add(P.nrow * sizeof(double));
    P.off_dz = L.add(g->nz * sizeof(double));
    P.off_dzc = L.add((g->nz + 1) * sizeof(double));
    P.off_cumh = L.add((g->nz + 1) * sizeof(double));
    P.off_tref = L.add(g->nz * sizeof(double));
    P.off_dtr = L.add(g->nz * 4 * P.esize);
    P.off_tab = L.add((size_t)4 * g->nz * P.esize);
    if (salinity) {
        P.off_sref = L.add(g->nz * sizeof(double));
        P.off_dsr = L.add(g->nz * 4 * P.esize);
        P.off_eos = L.add(g->nz * 2 * P.esize);
        P.off_zc = L.add(g->nz * sizeof(double));
    }
    P.off_part = L.add(P.diag_blocks * ocn::DG_COUNT * sizeof(double));
    P.off_out = L.add(ocn::DG_COUNT * sizeof(double));
    P.off_bw = L.add((size_t)(2 * ocn::baro_substeps(std::max(n_substeps, 1)) + 1) * sizeof(double));
    P.total = L.total;
    return P;
}

// Substep weights of the barotropic window: a_q proportional to cos^2(pi t),
// t = q/Ns - 1, on |t| < 1/2 (q = 1..M, M = Ns + Ns/2), normalised to sum to
// one; A_l = sum_{q>l} a_q for l = 0..M-1.
int upload_substep_weights(ocn_state* s) {
    const int ns = s->p.n_substeps, M = s->d.baro_m;
    std::vector<double> w(2 * (size_t)M + 1, 0.0);
    double sum = 0.0;
    for (int q = 1; q <= M; ++q) {
        const double t = double(q) / ns - 1.0;
        const double c = std::fabs(t) < 0.5 ? std::cos(3.14159265358979323846 * t) : 0.0;
        w[q] = c * c;
        sum += w[q];
    }
    for (int q = 1; q <= M; ++q) w[q] /= sum;
    double tail = 0.0;
    for (int l = M - 1; l >= 0; --l) {
        tail += w[l + 1];
        w[M + 1 + l] = tail;
    }
    HIPCHK(hipMemcpyAsync(s->d.baro_a, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return OCN_OK;
}

bool valid_params(const ocn_params* p, std::string& why) {
    if (!p) { why = "params is NULL"; return false; }
    if (p->precision != OCN_FP64 && p->precision != OCN_FP32) { why = "precision must be OCN_FP64 or OCN_FP32"; return false; }
    if (p->n_substeps < 1) { why = "n_substeps must be >= 1"; return false; }
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) { why = "dt must be positive"; return false; }
    if (!(p->kappa >= 0.0)) { why = "kappa must be >= 0"; return false; }
    if (!(p->rho0 > 0.0)) { why = "rho0 must be positive"; return false; }
    if (!(p->g > 0.0)) { why = "g must be positive"; return false; }
    {
        const double v[] = {p->chi, p->g, p->alpha, p->rho0, p->t_ref, p->kappa, p->restore_tau};
        for (double x : v)
            if (!std::isfinite(x)) { why = "chi, g, alpha, rho0, t_ref, kappa and restore_tau must be finite"; return false; }
    }
    if (p->baro_fuse < 0 || p->baro_fuse > 8) { why = "baro_fuse must be in 0..8"; return false; }
    if (p->salinity != 0 && p->salinity != 1) { why = "salinity must be 0 or 1"; return false; }
    if (p->salinity)
        for (int q = 0; q < 9; ++q)
            if (!std::isfinite(p->eos[q])) { why = "eos coefficients must be finite"; return false; }
    if (!(p->pgf_weight >= 0.0 && p->pgf_weight <= 1.0)) { why = "pgf_weight must be in [0, 1]"; return false; }
    if (p->momentum_form != 0 && p->momentum_form != 1) { why = "momentum_form must be 0 or 1"; return false; }
    if (p->reserved2 != 0) { why = "reserved2 must be 0"; return false; }
    return true;
}

// Fill a padded host image of a 3D field from interior doubles (periodic halo
// copies, zero beyond walls).
template <typename R>
void pack3(const ocn_state* s, const double* src, const double* sub_per_level, std::vector<R>& out) {
    const ocn_grid* g = s->g;
    const int nx = g->nx, ny = g->ny, nz = g->nz, h = g->h;
    const size_t p3 = s->d.p3, rows = ny + 2 * h;
    out.assign(s->n3, R(0));
    for (int k = 0; k < nz; ++k)
        for (int jj = -h; jj < ny + h; ++jj) {
            const int j = wrap(jj, ny, g->d.periodic_y);
            if (j < 0) continue;
            R* dst = out.data() + ((size_t)k * rows + (jj + h)) * p3 + s->ox3;
            const double* row = src + ((size_t)k * ny + j) * nx;
            const double sub = sub_per_level ? sub_per_level[k] : 0.0;
            for (int ii = -h; ii < nx + h; ++ii) {
                const int i = wrap(ii, nx, g->d.periodic_x);
                if (i < 0) continue;
                dst[ii] = R(row[i] - sub);
            }
        }
}

template <typename R>
void unpack3(const ocn_state* s, const std::vector<R>& img, const double* add_per_level, double* dst, int nlev) {
    const ocn_grid* g = s->g;
    const int nx = g->nx, ny = g->ny, h = g->h;
    const size_t p3 = s->d.p3, rows = ny + 2 * h;
    for (int k = 0; k < nlev; ++k)
        for (int j = 0; j < ny; ++j) {
            const R* row = img.data() + ((size_t)k * rows + (j + h)) * p3 + s->ox3;
            const double add = add_per_level ? add_per_level[k] : 0.0;
            for (int i = 0; i < nx; ++i) dst[((size_t)k * ny + j) * nx + i] = double(row[i]) + add;
        }
}

void pack2(const ocn_state* s, const double* src, std::vector<double>& out) {
    const ocn_grid* g = s->g;
    const int nx = g->nx, ny = g->ny, h = g->h;
    const size_t p2 = s->d.p2;
    out.assign(s->n2, 0.0);
    for (int jj = -h; jj < ny + h; ++jj) {
        const int j = wrap(jj, ny, g->d.periodic_y);
        if (j < 0) continue;
        for (int ii = -h; ii < nx + h; ++ii) {
            const int i = wrap(ii, nx, g->d.periodic_x);
            if (i < 0) continue;
            out[(size_t)(jj + h) * p2 + s->ox2 + ii] = src[(size_t)j * nx + i];
        }
    }
}

void unpack2(const ocn_state* s, const std::vector<double>& img, double* dst) {
    const ocn_grid* g = s->g;
    const int nx = g->nx, ny = g->ny, h = g->h;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) dst[(size_t)j * nx + i] = img[(size_t)(j + h) * s->d.p2 + s->ox2 + i];
}

// Device base address (padded origin) of a 3D or 2D array from its interior pointer.
void* base3(const ocn_state* s, void* interior) {
    return static_cast<unsigned char*>(interior) - ((size_t)s->g->h * s->d.p3 + s->ox3) * s->esize;
}
double* base2(const ocn_state* s, double* interior) { return interior - ((size_t)s->g->h * s->d.p2 + s->ox2); }

int kb_at(const ocn_grid* g, int i, int j) {
    const int ii = wrap(i, g->nx, g->d.periodic_x), jj = wrap(j, g->ny, g->d.periodic_y);
    if (ii < 0 || jj < 0) return 0;
    return g->kb[(size_t)jj * g->nx + ii];
}

template <typename R>
int upload_tables(ocn_state* s) {
    const ocn_grid* g = s->g;
    const int nz = g->nz;
    // reference-profile steps
    std::vector<R> dtr(nz * 4, R(0));
    const int offs[4] = {-2, -1, 1, 2};
    for (int k = 0; k < nz; ++k)
        for (int q = 0; q < 4; ++q) {
            const int l = k + offs[q];
            dtr[k * 4 + q] = (l >= 0 && l < nz) ? R(s->tref[l] - s->tref[k]) : R(0);
        }
    HIPCHK(hipMemcpyAsync(s->d.dtr, dtr.data(), dtr.size() * sizeof(R), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->d.tref, s->tref.data(), nz * sizeof(double), hipMemcpyHostToDevice, s->st));
    // restoring target as an anomaly of the top layer
    std::vector<double> ts(s->tstar.size());
    for (size_t c = 0; c < ts.size(); ++c) ts[c] = s->tstar[c] - s->tref[nz - 1];
    std::vector<double> img;
    pack2(s, ts.data(), img);
    HIPCHK(hipMemcpyAsync(base2(s, s->d.tstar), img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    if (!s->d.salinity) return OCN_OK;
    // salinity: reference steps, restoring target anomaly and the per-level
    // buoyancy coefficients of anomalies. With Ta = tref - t0 + T',
    // Sa = sref - s0 + S', the density anomaly relative to the reference water
    // of the level is T' (cT - a0 lambda1 T'/2 - nu S') + S' (cS - b0 lambda2 S'/2)
    // with cT = -a0 (1 + mu1 z + lambda1 (tref - t0)) - nu (sref - s0) and
    // cS = b0 (1 - mu2 z - lambda2 (sref - s0)) - nu (tref - t0); b' = -g rho'/rho0.
    std::vector<R> dsr(nz * 4, R(0));
    for (int k = 0; k < nz; ++k)
        for (int q = 0; q < 4; ++q) {
            const int l = k + offs[q];
            dsr[k * 4 + q] = (l >= 0 && l < nz) ? R(s->sref[l] - s->sref[k]) : R(0);
        }
    const double* e = s->d.eos;
    const double gr = s->p.g / s->p.rho0;
    std::vector<R> tab(nz * 2);
    std::vector<double> zc(nz);
    double depth = 0.0;
    for (int k = nz - 1; k >= 0; --k) {
        zc[k] = depth + 0.5 * g->dz[k];
        depth += g->dz[k];
    }
    for (int k = 0; k < nz; ++k) {
        const double ta = s->tref[k] - e[7], sa = s->sref[k] - e[8];
        const double cT = -e[0] * (1.0 + e[4] * zc[k] + e[2] * ta) - e[6] * sa;
        const double cS = e[1] * (1.0 - e[5] * zc[k] - e[3] * sa) - e[6] * ta;
        tab[2 * k] = R(-gr * cT);
        tab[2 * k + 1] = R(-gr * cS);
    }
    std::vector<double> ss(s->sstar.size());
    for (size_t c = 0; c < ss.size(); ++c) ss[c] = s->sstar[c] - s->sref[nz - 1];
    pack2(s, ss.data(), img);
    HIPCHK(hipMemcpyAsync(s->d.dsr, dsr.data(), dsr.size() * sizeof(R), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->d.sref, s->sref.data(), nz * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->d.eos_tab, tab.data(), tab.size() * sizeof(R), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->d.zc, zc.data(), nz * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(base2(s, s->d.sstar), img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return OCN_OK;
}

// The per-level reference of a tracer's stored anomaly: the mean over the wet
// cells of each level of the first field set.
void level_means(const ocn_grid* g, const double* host, std::vector<double>& ref) {
    const int nz = g->nz;
    const size_t n2 = (size_t)g->nx * g->ny;
    for (int k = 0; k < nz; ++k) {
        double sum = 0.0, all = 0.0;
        size_t n = 0;
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                const double v = host[(size_t)k * n2 + (size_t)j * g->nx + i];
                all += v;
                if (g->kb[(size_t)j * g->nx + i] >= nz - k) { sum += v; ++n; }
            }
        ref[k] = n ? sum / n : all / n2;
    }
}

template <typename R>
int init_static(ocn_state* s) {
    const ocn_grid* g = s->g;
    const int nx = g->nx, ny = g->ny, nz = g->nz, h = g->h;
    DevState& d = s->d;
    // wet-layer counts with a halo of hk = h + 1
    const int hk = d.hk;
    std::vector<int32_t> kbimg((size_t)d.pk * (ny + 2 * hk), 0);
    for (int j = -hk; j < ny + hk; ++j)
        for (int i = -hk; i < nx + hk; ++i) kbimg[(size_t)(j + hk) * d.pk + s->oxk + i] = kb_at(g, i, j);
    HIPCHK(hipMemcpyAsync(d.kb - ((size_t)hk * d.pk + s->oxk), kbimg.data(), kbimg.size() * 4, hipMemcpyHostToDevice, s->st));
    // row metrics
    const size_t nr = ny + 2 * h + 1;
    double* rows[6] = {d.dxc, d.dxv, d.area, d.fcor, d.metric, d.fcor_s};
    const std::vector<double>* src[6] = {&g->dxc, &g->dxv, &g->area, &g->fcor, &g->metric, &g->fcor_s};
    for (int q = 0; q < 6; ++q)
        HIPCHK(hipMemcpyAsync(rows[q] - h, src[q]->data(), nr * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(d.dz, g->dz.data(), nz * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(d.dzc, g->dzc.data(), (nz + 1) * sizeof(double), hipMemcpyHostToDevice, s->st));
    // column depths of u and v points (sum of wet layer thicknesses, bottom to top)
    std::vector<double> hu((size_t)nx * ny), hv((size_t)nx * ny);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int Ku = std::min(kb_at(g, i, j), kb_at(g, i - 1, j));
            const int Kv = std::min(kb_at(g, i, j), kb_at(g, i, j - 1));
            double a = 0.0, b = 0.0;
            for (int k = 0; k < nz; ++k) {
                if (k >= nz - Ku) a += g->dz[k];
                if (k >= nz - Kv) b += g->dz[k];
            }
            hu[(size_t)j * nx + i] = a;
            hv[(size_t)j * nx + i] = b;
        }
    // the same sums per wet-layer count (the fused barotropic kernel looks
    // depths up from the counts instead of reading hu, hv)
    std::vector<double> cumh(nz + 1);
    for (int K = 0; K <= nz; ++K) {
        double a = 0.0;
        for (int k = 0; k < nz; ++k)
            if (k >= nz - K) a += g->dz[k];
        cumh[K] = a;
    }
    HIPCHK(hipMemcpyAsync(d.cumh, cumh.data(), (nz + 1) * sizeof(double), hipMemcpyHostToDevice, s->st));
    std::vector<double> img;
    pack2(s, hu.data(), img);
    HIPCHK(hipMemcpyAsync(base2(s, d.hu), img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    pack2(s, hv.data(), img);
    HIPCHK(hipMemcpyAsync(base2(s, d.hv), img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    // Constant-diffusivity solve, eliminated from the surface down: the pivots
    // of the layers above a column's bottom do not depend on its depth, so one
    // level table serves every column; only the bottom layer's pivot differs,
    // and it is tabulated per level too.
    const double dt = s->p.dt, kap = s->p.kappa;
    std::vector<double> a(nz + 1, 0.0), c(nz, 0.0), bp(nz, 0.0);
    for (int k = 1; k < nz; ++k) a[k] = -dt * kap / g->dzc[k];  // face k (a[0], a[nz]: no interior face)
    for (int k = 0; k + 1 < nz; ++k) c[k] = a[k + 1];
    for (int k = nz - 1; k >= 0; --k) {
        const double b = g->dz[k] - a[k] - c[k];
        bp[k] = (k == nz - 1) ? b : b - c[k] * a[k + 1] / bp[k + 1];
    }
    std::vector<R> tab((size_t)4 * nz);
    for (int k = 0; k < nz; ++k) {
        const double above = (k + 1 < nz) ? c[k] * a[k + 1] / bp[k + 1] : 0.0;
        tab[4 * k + 0] = R(1.0 / bp[k]);
        tab[4 * k + 1] = R((k + 1 < nz) ? c[k] / bp[k + 1] : 0.0);
        tab[4 * k + 2] = R(1.0 / ((g->dz[k] - c[k]) - above));  // layer k as the bottom layer
        tab[4 * k + 3] = R(a[k]);
    }
    HIPCHK(hipMemcpyAsync(d.thomas_tab, tab.data(), tab.size() * sizeof(R), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return upload_tables<R>(s);
}

template <typename R>
int set3(ocn_state* s, void* interior, const double* host, const double* sub, int mask_kind) {
    const ocn_grid* g = s->g;
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    std::vector<double> tmp;
    const double* src = host;
    if (mask_kind) {  // zero dry velocity points
        tmp.assign(host, host + (size_t)nx * ny * nz);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int K = mask_kind == 1 ? std::min(kb_at(g, i, j), kb_at(g, i - 1, j))
                                             : std::min(kb_at(g, i, j), kb_at(g, i, j - 1));
                for (int k = 0; k < nz - K; ++k) tmp[((size_t)k * ny + j) * nx + i] = 0.0;
            }
        src = tmp.data();
    }
    std::vector<R> img;
    pack3<R>(s, src, sub, img);
    HIPCHK(hipMemcpyAsync(base3(s, interior), img.data(), img.size() * sizeof(R), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return OCN_OK;
}

template <typename R>
int get3(ocn_state* s, void* interior, double* host, const double* add, int nlev) {
    std::vector<R> img(s->n3);
    HIPCHK(hipMemcpyAsync(img.data(), base3(s, interior), img.size() * sizeof(R), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    unpack3<R>(s, img, add, host, nlev);
    return OCN_OK;
}

int set2(ocn_state* s, double* interior, const double* host) {
    std::vector<double> img;
    pack2(s, host, img);
    HIPCHK(hipMemcpyAsync(base2(s, interior), img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return OCN_OK;
}

int get2(ocn_state* s, double* interior, double* host) {
    std::vector<double> img(s->n2);
    HIPCHK(hipMemcpyAsync(img.data(), base2(s, interior), img.size() * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    unpack2(s, img, host);
    return OCN_OK;
}

template <typename R>
int set_field_t(ocn_state* s, int32_t f, const double* host) {
    const ocn_grid* g = s->g;
    const int nz = g->nz;
    DevState& d = s->d;
    switch (f) {
    case OCN_FIELD_U:
    case OCN_FIELD_V: {
        int rc = set3<R>(s, f == OCN_FIELD_U ? d.u : d.v, host, nullptr, f == OCN_FIELD_U ? 1 : 2);
        if (rc) return rc;
        HIPCHK(ocn::launch_colsum<R>(d, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        return OCN_OK;
    }
    case OCN_FIELD_T: {
        if (!s->t_set) {
            // reference profile: mean of T over the wet cells of each level
            level_means(g, host, s->tref);
            s->t_set = true;
            int rc = upload_tables<R>(s);
            if (rc) return rc;
        }
        return set3<R>(s, d.t, host, s->tref.data(), 0);
    }
    case OCN_FIELD_S:
    case OCN_FIELD_S_PRED:
    case OCN_FIELD_GS_PREV:
    case OCN_FIELD_SSTAR:
    case OCN_FIELD_SREF: {
        if (!d.salinity) return fail(OCN_E_STATE, "the state carries no salinity");
        if (f == OCN_FIELD_S) {
            if (!s->s_set) {
                level_means(g, host, s->sref);
                s->s_set = true;
                int rc = upload_tables<R>(s);
                if (rc) return rc;
            }
            return set3<R>(s, d.s, host, s->sref.data(), 0);
        }
        if (f == OCN_FIELD_S_PRED) {
            if (!s->s_set) return fail(OCN_E_STATE, "set S first: S_PRED is stored relative to S's reference profile");
            return set3<R>(s, d.ss, host, s->sref.data(), 0);
        }
        if (f == OCN_FIELD_GS_PREV) return set3<R>(s, d.gs, host, nullptr, 0);
        if (f == OCN_FIELD_SSTAR) {
            s->sstar.assign(host, host + (size_t)g->nx * g->ny);
            return upload_tables<R>(s);
        }
        if (s->s_set) return fail(OCN_E_STATE, "SREF can only be set before S");
        s->sref.assign(host, host + nz);
        return upload_tables<R>(s);
    }
    case OCN_FIELD_GU_PREV: return set3<R>(s, d.gu, host, nullptr, 0);
    case OCN_FIELD_GV_PREV: return set3<R>(s, d.gv, host, nullptr, 0);
    case OCN_FIELD_GT_PREV: return set3<R>(s, d.gt, host, nullptr, 0);
    case OCN_FIELD_U_PRED: return set3<R>(s, d.us, host, nullptr, 0);
    case OCN_FIELD_V_PRED: return set3<R>(s, d.vs, host, nullptr, 0);
    case OCN_FIELD_T_PRED:
        if (!s->t_set) return fail(OCN_E_STATE, "set T first: T_PRED is stored relative to T's reference profile");
        return set3<R>(s, d.ts, host, s->tref.data(), 0);
    case OCN_FIELD_GU_SLOW: return set2(s, d.gU, host);
    case OCN_FIELD_GV_SLOW: return set2(s, d.gV, host);
    case OCN_FIELD_ETA: return set2(s, d.eta, host);
    case OCN_FIELD_UBT: return set2(s, d.ubt, host);
    case OCN_FIELD_VBT: return set2(s, d.vbt, host);
    case OCN_FIELD_ETA_MEAN: return set2(s, d.eta_mean, host);
    case OCN_FIELD_UBT_MEAN: return set2(s, d.ubt_mean, host);
    case OCN_FIELD_VBT_MEAN: return set2(s, d.vbt_mean, host);
    case OCN_FIELD_TAUX: return set2(s, d.taux, host);
    case OCN_FIELD_TAUY: return set2(s, d.tauy, host);
    case OCN_FIELD_TSTAR: {
        s->tstar.assign(host, host + (size_t)g->nx * g->ny);
        return upload_tables<R>(s);
    }
    case OCN_FIELD_KAPPA: {
        if (!s->closure || s->net) return fail(OCN_E_STATE, "KAPPA is set only with a prescribed-field closure attached");
        return set3<R>(s, d.kw, host, nullptr, 0);
    }
    case OCN_FIELD_TREF: {
        if (s->t_set) return fail(OCN_E_STATE, "TREF can only be set before T");
        s->tref.assign(host, host + nz);
        return upload_tables<R>(s);
    }
    default: return fail(OCN_E_INVALID, "field cannot be set");
    }
}

template <typename R>
int get_field_t(ocn_state* s, int32_t f, double* host) {
    DevState& d = s->d;
    const ocn_grid* g = s->g;
    switch (f) {
    case OCN_FIELD_U: return get3<R>(s, d.u, host, nullptr, g->nz);
    case OCN_FIELD_V: return get3<R>(s, d.v, host, nullptr, g->nz);
    case OCN_FIELD_T: return get3<R>(s, d.t, host, s->tref.data(), g->nz);
    case OCN_FIELD_GU_PREV: return get3<R>(s, d.gu, host, nullptr, g->nz);
    case OCN_FIELD_GV_PREV: return get3<R>(s, d.gv, host, nullptr, g->nz);
    case OCN_FIELD_GT_PREV: return get3<R>(s, d.gt, host, nullptr, g->nz);
    case OCN_FIELD_U_PRED: return get3<R>(s, d.us, host, nullptr, g->nz);
    case OCN_FIELD_V_PRED: return get3<R>(s, d.vs, host, nullptr, g->nz);
    case OCN_FIELD_T_PRED: return get3<R>(s, d.ts, host, s->tref.data(), g->nz);
    case OCN_FIELD_GU_SLOW: return get2(s, d.gU, host);
    case OCN_FIELD_GV_SLOW: return get2(s, d.gV, host);
    case OCN_FIELD_S:
    case OCN_FIELD_S_PRED:
    case OCN_FIELD_GS_PREV:
    case OCN_FIELD_SSTAR:
    case OCN_FIELD_SREF:
        if (!d.salinity) return fail(OCN_E_STATE, "the state carries no salinity");
        if (f == OCN_FIELD_S) return get3<R>(s, d.s, host, s->sref.data(), g->nz);
        if (f == OCN_FIELD_S_PRED) return get3<R>(s, d.ss, host, s->sref.data(), g->nz);
        if (f == OCN_FIELD_GS_PREV) return get3<R>(s, d.gs, host, nullptr, g->nz);
        if (f == OCN_FIELD_SSTAR) {
            std::copy(s->sstar.begin(), s->sstar.end(), host);
            return OCN_OK;
        }
        std::copy(s->sref.begin(), s->sref.end(), host);
        return OCN_OK;
    case OCN_FIELD_ETA: return get2(s, d.eta, host);
    case OCN_FIELD_UBT: return get2(s, d.ubt, host);
    case OCN_FIELD_VBT: return get2(s, d.vbt, host);
    case OCN_FIELD_ETA_MEAN: return get2(s, d.eta_mean, host);
    case OCN_FIELD_UBT_MEAN: return get2(s, d.ubt_mean, host);
    case OCN_FIELD_VBT_MEAN: return get2(s, d.vbt_mean, host);
    case OCN_FIELD_TAUX: return get2(s, d.taux, host);
    case OCN_FIELD_TAUY: return get2(s, d.tauy, host);
    case OCN_FIELD_TSTAR: {
        std::copy(s->tstar.begin(), s->tstar.end(), host);
        return OCN_OK;
    }
    case OCN_FIELD_TREF: {
        std::copy(s->tref.begin(), s->tref.end(), host);
        return OCN_OK;
    }
    case OCN_FIELD_KAPPA: {  // tracer diffusivity on every z-face, 0 where the face is dry
        const int nx = g->nx, ny = g->ny, nz = g->nz;
        if (s->closure) {
            int rc = get3<R>(s, d.kw, host, nullptr, nz);
            if (rc) return rc;
        }
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    double& v = host[((size_t)k * ny + j) * nx + i];
                    const bool wet = k > nz - kb_at(g, i, j);
                    if (!s->closure) v = s->p.kappa;
                    if (!wet) v = 0.0;
                }
        return OCN_OK;
    }
    case OCN_FIELD_VISC: {  // momentum coefficient on every tracer z-face, 0 where the face is dry
        const int nx = g->nx, ny = g->ny, nz = g->nz;
        if (s->closure) {
            int rc = get3<R>(s, d.kv ? d.kv : d.kw, host, nullptr, nz);
            if (rc) return rc;
        }
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    double& v = host[((size_t)k * ny + j) * nx + i];
                    const bool wet = k > nz - kb_at(g, i, j);
                    if (!s->closure) v = s->p.kappa;
                    if (!wet) v = 0.0;
                }
        return OCN_OK;
    }
    case OCN_FIELD_W: {
        // faces 0..nz-1 go to the tracer-history buffer the next step writes
        // (its contents are dead between steps), the surface face to 2D scratch
        DevState dw = d;
        dw.ts = d.gt_out;
        HIPCHK(ocn::launch_w_faces<R>(dw, nullptr, s->st));
        const size_t n2 = (size_t)g->nx * g->ny;
        int rc = get3<R>(s, d.gt_out, host, nullptr, g->nz);
        if (rc) return rc;
        return get2(s, d.scratch2d, host + (size_t)g->nz * n2);
    }
    default: return fail(OCN_E_INVALID, "unknown field");
    }
}

size_t field_count(const ocn_grid* g, int32_t f) {
    const size_t n2 = (size_t)g->nx * g->ny, n3 = n2 * g->nz;
    switch (f) {
    case OCN_FIELD_U: case OCN_FIELD_V: case OCN_FIELD_T: case OCN_FIELD_KAPPA: case OCN_FIELD_VISC:
    case OCN_FIELD_GU_PREV: case OCN_FIELD_GV_PREV: case OCN_FIELD_GT_PREV:
    case OCN_FIELD_U_PRED: case OCN_FIELD_V_PRED: case OCN_FIELD_T_PRED: return n3;
    case OCN_FIELD_GU_SLOW: case OCN_FIELD_GV_SLOW: return n2;
    case OCN_FIELD_S: case OCN_FIELD_S_PRED: case OCN_FIELD_GS_PREV: return n3;
    case OCN_FIELD_SSTAR: return n2;
    case OCN_FIELD_SREF: return g->nz;
    case OCN_FIELD_W: return n2 * (g->nz + 1);
    case OCN_FIELD_TREF: return g->nz;
    case OCN_FIELD_ETA: case OCN_FIELD_UBT: case OCN_FIELD_VBT: case OCN_FIELD_ETA_MEAN:
    case OCN_FIELD_UBT_MEAN: case OCN_FIELD_VBT_MEAN: case OCN_FIELD_TAUX: case OCN_FIELD_TAUY:
    case OCN_FIELD_TSTAR: return n2;
    default: return 0;
    }
}

}  // namespace

extern "C" {

uint32_t ocn_abi_version(void) { return OCN_ABI_VERSION; }

const char* ocn_last_error(void) { return g_err.c_str(); }

int ocn_grid_create(const ocn_grid_desc* desc, ocn_grid** out) {
    try {
        if (!desc || !out) return fail(OCN_E_INVALID, "desc and out must not be NULL");
        const ocn_grid_desc& d = *desc;
        if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(OCN_E_INVALID, "nx, ny, nz must be >= 1");
        if (d.halo < 3 || d.halo > 8) return fail(OCN_E_INVALID, "halo must be in 3..8");
        if (d.coords != OCN_CARTESIAN && d.coords != OCN_LATLON) return fail(OCN_E_INVALID, "bad coords");
        if (d.coords == OCN_LATLON && d.periodic_y) return fail(OCN_E_INVALID, "a lat-lon grid cannot be periodic in y");
        if (!d.dz) return fail(OCN_E_INVALID, "dz must not be NULL");
        if (!(d.dx > 0) || !(d.dy > 0)) return fail(OCN_E_INVALID, "dx and dy must be positive");
        if (d.reserved != 0) return fail(OCN_E_INVALID, "reserved must be 0");
        if (d.nz > 1024) return fail(OCN_E_UNSUPPORTED, "nz above 1024");
        if (d.coords == OCN_LATLON) {
            const double south = d.y0 - d.halo * d.dy, north = d.y0 + (d.ny + d.halo) * d.dy;
            if (south <= -90.0 || north >= 90.0) return fail(OCN_E_INVALID, "lat-lon grid and halo must stay inside (-90, 90)");
        }
        for (int k = 0; k < d.nz; ++k)
            if (!(d.dz[k] > 0)) return fail(OCN_E_INVALID, "dz must be positive");
        ocn_grid* g = new ocn_grid();
        g->d = d;
        g->d.dz = nullptr;
        g->d.kbottom = nullptr;
        g->nx = d.nx; g->ny = d.ny; g->nz = d.nz; g->h = d.halo;
        g->dz.assign(d.dz, d.dz + d.nz);
        g->dzc.assign(d.nz + 1, 0.0);
        for (int k = 1; k < d.nz; ++k) g->dzc[k] = 0.5 * (d.dz[k - 1] + d.dz[k]);
        g->kb.assign((size_t)d.nx * d.ny, d.nz);
        if (d.kbottom)
            for (size_t c = 0; c < g->kb.size(); ++c) g->kb[c] = std::max(0, std::min<int32_t>(d.nz, d.kbottom[c]));
        const int nr = d.ny + 2 * d.halo + 1;
        g->dxc.resize(nr); g->dxv.resize(nr); g->area.resize(nr); g->fcor.resize(nr); g->metric.resize(nr);
        g->fcor_s.resize(nr);
        const double rad = kPi / 180.0;
        g->dy = d.coords == OCN_LATLON ? d.radius * d.dy * rad : d.dy;
        for (int q = 0; q < nr; ++q) {
            int j = q - d.halo;
            if (d.periodic_y) j = wrap(j, d.ny, true);
            if (d.coords == OCN_LATLON) {
                const double latc = d.y0 + (j + 0.5) * d.dy, lats = d.y0 + j * d.dy;
                g->dxc[q] = d.radius * std::cos(latc * rad) * (d.dx * rad);
                g->dxv[q] = d.radius * std::cos(lats * rad) * (d.dx * rad);
                g->fcor[q] = 2.0 * d.omega * std::sin(latc * rad);
                g->fcor_s[q] = 2.0 * d.omega * std::sin(lats * rad);
                g->metric[q] = std::tan(latc * rad) / d.radius;
            } else {
                g->dxc[q] = d.dx;
                g->dxv[q] = d.dx;
                g->fcor[q] = d.f0 + d.beta * ((j + 0.5) * d.dy - 0.5 * d.ny * d.dy);
                g->fcor_s[q] = d.f0 + d.beta * (j * d.dy - 0.5 * d.ny * d.dy);
                g->metric[q] = 0.0;
            }
            g->area[q] = g->dxc[q] * g->dy;
        }
        *out = g;
        return OCN_OK;
    } catch (const std::bad_alloc&) {
        return fail(OCN_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(OCN_E_INVALID, "unexpected error");
    }
}

void ocn_grid_destroy(ocn_grid* grid) { delete grid; }

int ocn_state_arena_bytes(const ocn_grid* grid, const ocn_params* params, size_t* bytes) {
    if (!grid || !bytes) return fail(OCN_E_INVALID, "grid and bytes must not be NULL");
    std::string why;
    if (!valid_params(params, why)) return fail(OCN_E_INVALID, why);
    if (grid->nz > ocn::kMaxLevels) return fail(OCN_E_UNSUPPORTED, "nz above 128 is not supported (column solve, tendency level table)");
    *bytes = make_plan(grid, params->precision, params->n_substeps, params->salinity).total;
    return OCN_OK;
}

int ocn_state_init(const ocn_grid* grid, const ocn_params* params, void* device_arena, size_t arena_bytes,
                   void* hip_stream, ocn_state** out) {
    try {
        if (!grid || !out || !device_arena) return fail(OCN_E_INVALID, "grid, arena and out must not be NULL");
        std::string why;
        if (!valid_params(params, why)) return fail(OCN_E_INVALID, why);
        if (reinterpret_cast<uintptr_t>(device_arena) % 256) return fail(OCN_E_INVALID, "arena must be 256-byte aligned");
        const Plan P = make_plan(grid, params->precision, params->n_substeps, params->salinity);
        if (arena_bytes < P.total) return fail(OCN_E_NOMEM, "arena smaller than ocn_state_arena_bytes");
        if (grid->nz > ocn::kMaxLevels) return fail(OCN_E_UNSUPPORTED, "nz above 128 is not supported (column solve, tendency level table)");

        ocn_state* s = new ocn_state();
        s->g = grid;
        s->p = *params;
        s->st = static_cast<hipStream_t>(hip_stream);
        s->arena = device_arena;
        s->bytes = arena_bytes;
        s->esize = (int)P.esize;
        s->ox3 = P.ox3; s->ox2 = P.ox2; s->oxk = P.oxk;
        s->n3 = P.n3; s->n2 = P.n2; s->nk = P.nk;
        s->tref.assign(grid->nz, 0.0);
        s->tstar.assign((size_t)grid->nx * grid->ny, 0.0);

        unsigned char* A = static_cast<unsigned char*>(device_arena);
        DevState& d = s->d;
        const int h = grid->h;
        d.nx = grid->nx; d.ny = grid->ny; d.nz = grid->nz; d.h = h;
        d.hk = h + 1;
        d.periodic_x = grid->d.periodic_x ? 1 : 0;
        d.periodic_y = grid->d.periodic_y ? 1 : 0;
        d.latlon = grid->d.coords == OCN_LATLON;
        d.p3 = (int)P.p3; d.p2 = (int)P.p2; d.pk = (int)P.pk;
        d.ox2 = (int)P.ox2;
        d.plane3 = (long long)P.p3 * (long long)P.rows;
        const size_t o3 = ((size_t)h * P.p3 + P.ox3) * P.esize;
        void** f3s[14] = {&d.u, &d.v, &d.t, &d.us, &d.vs, &d.ts, &d.gu, &d.gv, &d.gt, &d.gt_out,
                          &d.s, &d.ss, &d.gs, &d.gs_out};
        for (int q = 0; q < P.nf3; ++q) *f3s[q] = A + P.off_f3[q] + o3;
        s->gtb[0] = d.gt;
        s->gtb[1] = d.gt_out;
        double** f2s[25] = {&d.eta, &d.ubt, &d.vbt, &d.se, &d.su, &d.sv, &d.eta_mean, &d.ubt_mean, &d.vbt_mean,
                            &d.gU, &d.gV, &d.hu, &d.hv, &d.cu, &d.cv, &d.taux, &d.tauy, &d.tstar, &d.scratch2d,
                            &d.eta2, &d.ubt2, &d.vbt2, &d.sfu, &d.sfv, &d.sstar};
        const size_t o2 = (size_t)h * P.p2 + P.ox2;
        for (int q = 0; q < P.nf2; ++q) *f2s[q] = reinterpret_cast<double*>(A + P.off_f2[q]) + o2;
        d.salinity = params->salinity;
        if (d.salinity) {
            d.sref = reinterpret_cast<double*>(A + P.off_sref);
            d.dsr = A + P.off_dsr;
            d.eos_tab = A + P.off_eos;
            d.zc = reinterpret_cast<double*>(A + P.off_zc);
            for (int q = 0; q < 9; ++q) d.eos[q] = params->eos[q];
            const double gr = params->g / params->rho0;
            d.eos_qT = gr * 0.5 * params->eos[0] * params->eos[2];
            d.eos_qTS = gr * params->eos[6];
            d.eos_qS = gr * 0.5 * params->eos[1] * params->eos[3];
            s->sref.assign(grid->nz, 0.0);
            s->sstar.assign((size_t)grid->nx * grid->ny, 0.0);
        }
        d.kb = reinterpret_cast<int*>(A + P.off_kb) + ((size_t)(h + 1) * P.pk + P.oxk);
        double** rows[6] = {&d.dxc, &d.dxv, &d.area, &d.fcor, &d.metric, &d.fcor_s};
        for (int q = 0; q < 6; ++q) *rows[q] = reinterpret_cast<double*>(A + P.off_rows[q]) + h;
        d.dy = grid->dy;
        d.dz = reinterpret_cast<double*>(A + P.off_dz);
        d.dzc = reinterpret_cast<double*>(A + P.off_dzc);
        d.cumh = reinterpret_cast<double*>(A + P.off_cumh);
        d.tref = reinterpret_cast<double*>(A + P.off_tref);
        d.dtr = A + P.off_dtr;
        d.thomas_tab = A + P.off_tab;
        d.diag_part = reinterpret_cast<double*>(A + P.off_part);
        d.diag_out = reinterpret_cast<double*>(A + P.off_out);
        d.diag_blocks = (int)P.diag_blocks;
        d.dt = params->dt;
        d.chi = params->chi;
        d.g = params->g;
        d.alpha = params->alpha;
        d.rho0 = params->rho0;
        d.kappa = params->kappa;
        d.restore_inv = params->restore_tau > 0.0 ? 1.0 / params->restore_tau : 0.0;
        d.pgf_w = params->pgf_weight;
        d.vi = params->momentum_form;
        d.n_substeps = params->n_substeps;
        d.baro_fuse = params->baro_fuse == 0 ? ocn::kBaroFuseDefault : params->baro_fuse;
        d.baro_m = ocn::baro_substeps(params->n_substeps);
        d.baro_a = reinterpret_cast<double*>(A + P.off_bw);
        d.baro_A = d.baro_a + d.baro_m + 1;
        d.tend_ty = 0;

        hipError_t e = hipMemsetAsync(device_arena, 0, P.total, s->st);
        if (e == hipSuccess) e = hipStreamSynchronize(s->st);
        if (e != hipSuccess) {
            delete s;
            return fail(OCN_E_DEVICE, std::string("arena clear: ") + hipGetErrorString(e));
        }
        // barotropic CFL of a substep: sqrt(g H) dtau sqrt(1/dx^2 + 1/dy^2) over wet columns
        {
            const double dtau = params->dt / params->n_substeps;
            for (int j = 0; j < grid->ny; ++j) {
                const double dxc = grid->dxc[grid->row(j)];
                for (int i = 0; i < grid->nx; ++i) {
                    const int kb = grid->kb[(size_t)j * grid->nx + i];
                    if (kb <= 0) continue;
                    double hc = 0.0;
                    for (int k = grid->nz - kb; k < grid->nz; ++k) hc += grid->dz[k];
                    const double c = std::sqrt(params->g * hc) * dtau *
                                     std::sqrt(1.0 / (dxc * dxc) + 1.0 / (grid->dy * grid->dy));
                    s->cfl_bt = std::max(s->cfl_bt, c);
                }
            }
        }
        int rc = params->precision == OCN_FP32 ? init_static<float>(s) : init_static<double>(s);
        if (!rc) rc = upload_substep_weights(s);
        if (rc) {
            delete s;
            return rc;
        }
        *out = s;
        return OCN_OK;
    } catch (const std::bad_alloc&) {
        return fail(OCN_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(OCN_E_INVALID, "unexpected error");
    }
}

void ocn_state_destroy(ocn_state* state) {
    if (state) {
        (void)hipStreamSynchronize(state->st);
        drop_graph(state);
        drop_events(state);
        delete state;
    }
}

int ocn_set_field(ocn_state* s, int32_t field, const double* host, size_t count) {
    try {
        if (!s || !host) return fail(OCN_E_INVALID, "state and host must not be NULL");
        const size_t n = field_count(s->g, field);
        if (n == 0 || field == OCN_FIELD_W) return fail(OCN_E_INVALID, "field cannot be set");
        if (count != n) return fail(OCN_E_INVALID, "count does not match the field size");
        return s->esize == 4 ? set_field_t<float>(s, field, host) : set_field_t<double>(s, field, host);
    } catch (const std::bad_alloc&) {
        return fail(OCN_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(OCN_E_INVALID, "unexpected error");
    }
}

int ocn_get_field(ocn_state* s, int32_t field, double* host, size_t count) {
    try {
        if (!s || !host) return fail(OCN_E_INVALID, "state and host must not be NULL");
        const size_t n = field_count(s->g, field);
        if (n == 0) return fail(OCN_E_INVALID, "unknown field");
        if (count != n) return fail(OCN_E_INVALID, "count does not match the field size");
        return s->esize == 4 ? get_field_t<float>(s, field, host) : get_field_t<double>(s, field, host);
    } catch (const std::bad_alloc&) {
        return fail(OCN_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(OCN_E_INVALID, "unexpected error");
    }
}

int ocn_set_first_step(ocn_state* s, int32_t first) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    s->first = first ? 1 : 0;
    return OCN_OK;
}

int ocn_get_first_step(ocn_state* s, int32_t* first) {
    if (!s || !first) return fail(OCN_E_INVALID, "state and first must not be NULL");
    *first = s->first;
    return OCN_OK;
}


namespace {

// Learned closure: features of every column -> network -> face diffusivity.
int closure_update(ocn_state* s) {
    const bool f32 = s->esize == 4;
    const int rows = s->g->nx * s->g->ny;
    HIPCHK(f32 ? ocn::launch_features<float>(s->d, s->din, s->norm, s->xb, 1, s->st)
               : ocn::launch_features<double>(s->d, s->din, s->norm, s->xb, 1, s->st));
    HIPCHK(ocn::mlp_infer(s->net, s->xb, rows, s->h1b, s->h2b, s->y, s->st));
    HIPCHK(f32 ? ocn::launch_kappa_map<float>(s->d, s->y, s->dout, s->p.kappa, s->st)
               : ocn::launch_kappa_map<double>(s->d, s->y, s->dout, s->p.kappa, s->st));
    return OCN_OK;
}

struct ClosurePlan {
    size_t kw, kv, norm, xb, h1b, h2b, y, total;
};

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

ClosurePlan closure_plan(const ocn_state* s, int din, int h1, int h2, int dout) {
    ClosurePlan P{};
    const size_t rows = (size_t)s->g->nx * s->g->ny;
    size_t off = 0;
    auto add = [&](size_t b) { size_t o = off; off = up256(off + b); return o; };
    P.kw = add(s->n3 * s->esize);
    if (din == 0) P.kv = add(s->n3 * s->esize);  // viscosity of Richardson mixing (prescribed mode)
    if (din > 0) {
        P.norm = add((size_t)2 * din * sizeof(float));
        P.xb = add(rows * din * 2);
        P.h1b = add(rows * h1 * 2);
        P.h2b = add(rows * h2 * 2);
        P.y = add(rows * dout * sizeof(float));
    }
    P.total = off;
    return P;
}

}  // namespace

namespace {

// Enqueue the kernels of one stage on the state's stream. The tendency stage
// writes G^n of the tracer to the second history buffer, which then becomes
// the history the next step reads.
int enqueue_stage(ocn_state* s, int stage) {
    const bool f32 = s->esize == 4;
    switch (stage) {
    case OCN_STAGE_MIXING: {
        int rc;
        if (s->closure && s->net && (rc = closure_update(s))) return rc;
        if (s->closure && !s->net && s->ri_on)
            HIPCHK(f32 ? ocn::launch_richardson<float>(s->d, s->ri, s->st)
                       : ocn::launch_richardson<double>(s->d, s->ri, s->st));
        else if (s->closure && !s->net && s->kappa_conv > 0.0)
            HIPCHK(f32 ? ocn::launch_convective<float>(s->d, s->kappa_conv, s->p.kappa, s->st)
                       : ocn::launch_convective<double>(s->d, s->kappa_conv, s->p.kappa, s->st));
        return OCN_OK;
    }
    case OCN_STAGE_TENDENCY:
        HIPCHK(f32 ? ocn::launch_tendency<float>(s->d, s->first, s->st)
                   : ocn::launch_tendency<double>(s->d, s->first, s->st));
        s->swap_history();
        return OCN_OK;
    case OCN_STAGE_BAROTROPIC:
        HIPCHK(ocn::launch_barotropic(s->d, s->st));
        return OCN_OK;
    case OCN_STAGE_COLUMN:
        HIPCHK(f32 ? ocn::launch_column<float>(s->d, s->st) : ocn::launch_column<double>(s->d, s->st));
        return OCN_OK;
    default:
        return fail(OCN_E_INVALID, "unknown stage");
    }
}

// Enqueue the kernels of one step on the state's stream (no host bookkeeping
// beyond the history buffers).
int enqueue_step(ocn_state* s) {
    int rc;
    for (int stage = OCN_STAGE_MIXING; stage <= OCN_STAGE_COLUMN; ++stage) {
        if (s->timing && (rc = record(s))) return rc;
        if ((rc = enqueue_stage(s, stage))) return rc;
    }
    if (s->timing) {
        if ((rc = record(s))) return rc;
        s->timed_steps += 1;
    }
    return OCN_OK;
}

void advance(ocn_state* s) {
    s->first = 0;
    s->step += 1;
    s->time += s->p.dt;
}

}  // namespace

int ocn_step(ocn_state* s, int32_t n) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    if (n < 0) return fail(OCN_E_INVALID, "n must be >= 0");
    int rc;
    for (int q = 0; q < n; ++q) {
        if ((rc = enqueue_step(s))) return rc;
        advance(s);
    }
    return OCN_OK;
}

int ocn_step_graph(ocn_state* s, int32_t n) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    if (n < 0) return fail(OCN_E_INVALID, "n must be >= 0");
    if (!s->st) return fail(OCN_E_UNSUPPORTED, "graph stepping needs a stream other than the null stream");
    int rc;
    for (int q = 0; q < n; ++q) {
        if (s->first || s->timing) {  // the start step and timed steps run eagerly
            if ((rc = enqueue_step(s))) return rc;
        } else {
            const int par = s->parity();
            if (!s->exec[par]) {
                HIPCHK(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
                rc = enqueue_step(s);
                hipGraph_t g = nullptr;
                hipError_t ce = hipStreamEndCapture(s->st, &g);
                // the capture recorded the step without running it; its tendency
                // stage swapped the history buffers, which the replay below does
                if (s->parity() != par) s->swap_history();
                if (rc) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc;
                }
                if (ce != hipSuccess) return fail(OCN_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
                s->graph[par] = g;
                HIPCHK(hipGraphInstantiate(&s->exec[par], s->graph[par], nullptr, nullptr, 0));
            }
            HIPCHK(hipGraphLaunch(s->exec[par], s->st));
            s->swap_history();  // what the replayed tendency stage did
        }
        advance(s);
    }
    return OCN_OK;
}

int ocn_debug_run_stage(ocn_state* s, int32_t stage) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    if (stage < OCN_STAGE_MIXING || stage > OCN_STAGE_COLUMN) return fail(OCN_E_INVALID, "unknown stage");
    return enqueue_stage(s, stage);
}

int ocn_closure_workspace_bytes(const ocn_state* s, const ocn_mlp* net, size_t* bytes) {
    if (!s || !bytes) return fail(OCN_E_INVALID, "state and bytes must not be NULL");
    int din = 0, h1 = 0, h2 = 0, dout = 0;
    if (net) ocn::mlp_shape(net, &din, &h1, &h2, &dout);
    *bytes = closure_plan(s, din, h1, h2, dout).total;
    return OCN_OK;
}

int ocn_closure_attach(ocn_state* s, const ocn_mlp* net, const float* norm, size_t norm_count, void* workspace,
                       size_t bytes) {
    if (!s || !workspace) return fail(OCN_E_INVALID, "state and workspace must not be NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(OCN_E_INVALID, "workspace must be 256-byte aligned");
    const int nz = s->g->nz;
    if ((size_t)2 * nz * 32 * s->esize > 64 * 1024)  // the LDS-staged solve at 32 columns per workgroup
        return fail(OCN_E_UNSUPPORTED, "nz too large for the variable-diffusivity column solve");
    int din = 0, h1 = 0, h2 = 0, dout = 0;
    if (net) {
        if (s->d.salinity) return fail(OCN_E_UNSUPPORTED, "the closure network takes temperature-only states");
        ocn::mlp_shape(net, &din, &h1, &h2, &dout);
        if (dout != nz) return fail(OCN_E_INVALID, "network output width must equal nz");
        if (din < 4 * nz + 3) return fail(OCN_E_INVALID, "network input width must be at least 4 nz + 3");
        if (ocn::features_lds(din) > 64 * 1024) return fail(OCN_E_UNSUPPORTED, "network input too wide");
        if (!norm || norm_count != (size_t)2 * din) return fail(OCN_E_INVALID, "norm must hold 2 din values");
        for (int f = 0; f < din; ++f)
            if (!std::isfinite(norm[f]) || !(norm[din + f] > 0.f) || !std::isfinite(norm[din + f]))
                return fail(OCN_E_INVALID, "norm: means must be finite and deviations positive");
    }
    const ClosurePlan P = closure_plan(s, din, h1, h2, dout);
    if (bytes < P.total) return fail(OCN_E_NOMEM, "workspace smaller than ocn_closure_workspace_bytes");
    HIPCHK(hipStreamSynchronize(s->st));
    drop_graph(s);
    unsigned char* W = static_cast<unsigned char*>(workspace);
    const size_t o3 = ((size_t)s->g->h * s->d.p3 + s->ox3) * s->esize;
    HIPCHK(s->esize == 4 ? ocn::launch_fill<float>(W + P.kw, (long long)s->n3, s->p.kappa, s->st)
                         : ocn::launch_fill<double>(W + P.kw, (long long)s->n3, s->p.kappa, s->st));
    s->d.kw = W + P.kw + o3;
    s->d.kv = nullptr;
    s->kv_ws = net ? nullptr : W + P.kv + o3;
    s->ri_on = false;
    s->kappa_conv = 0.0;
    s->closure = true;
    s->net = net;
    s->din = din; s->h1 = h1; s->h2 = h2; s->dout = dout;
    if (net) {
        s->norm = reinterpret_cast<float*>(W + P.norm);
        s->xb = reinterpret_cast<uint16_t*>(W + P.xb);
        s->h1b = reinterpret_cast<uint16_t*>(W + P.h1b);
        s->h2b = reinterpret_cast<uint16_t*>(W + P.h2b);
        s->y = reinterpret_cast<float*>(W + P.y);
        HIPCHK(hipMemcpyAsync(s->norm, norm, (size_t)2 * din * sizeof(float), hipMemcpyHostToDevice, s->st));
    }
    HIPCHK(hipStreamSynchronize(s->st));
    return OCN_OK;
}

int ocn_closure_convective(ocn_state* s, double kappa_conv) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    if (!s->closure || s->net) return fail(OCN_E_STATE, "needs a prescribed-field closure attached");
    if (!std::isfinite(kappa_conv)) return fail(OCN_E_INVALID, "kappa_conv must be finite");
    HIPCHK(hipStreamSynchronize(s->st));
    drop_graph(s);
    s->kappa_conv = kappa_conv > 0.0 ? kappa_conv : 0.0;
    if (s->kappa_conv > 0.0) {  // replaces Richardson mixing: momentum uses the diffusivity again
        s->ri_on = false;
        s->d.kv = nullptr;
    }
    return OCN_OK;
}

int ocn_closure_richardson(ocn_state* s, double nu0, double alpha, double nu_b, double kappa_b, double conv) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    if (!s->closure || s->net || !s->kv_ws) return fail(OCN_E_STATE, "needs a prescribed-field closure attached");
    if (!std::isfinite(nu0) || !(alpha >= 0.0) || !(nu_b >= 0.0) || !(kappa_b >= 0.0) || !(conv >= 0.0) ||
        !std::isfinite(alpha) || !std::isfinite(nu_b) || !std::isfinite(kappa_b) || !std::isfinite(conv))
        return fail(OCN_E_INVALID, "constants must be finite; alpha, nu_b, kappa_b and conv >= 0");
    HIPCHK(hipStreamSynchronize(s->st));
    drop_graph(s);
    if (nu0 > 0.0) {
        s->ri_on = true;
        s->ri = ocn::RiParams{nu0, alpha, nu_b, kappa_b, conv};
        s->kappa_conv = 0.0;
        s->d.kv = s->kv_ws;
        HIPCHK(s->esize == 4 ? ocn::launch_richardson<float>(s->d, s->ri, s->st)
                             : ocn::launch_richardson<double>(s->d, s->ri, s->st));
    } else {  // off: the constant diffusivity on every face, momentum with it
        s->ri_on = false;
        s->d.kv = nullptr;
        const size_t o3 = ((size_t)s->g->h * s->d.p3 + s->ox3) * s->esize;
        unsigned char* base = static_cast<unsigned char*>(s->d.kw) - o3;
        HIPCHK(s->esize == 4 ? ocn::launch_fill<float>(base, (long long)s->n3, s->p.kappa, s->st)
                             : ocn::launch_fill<double>(base, (long long)s->n3, s->p.kappa, s->st));
    }
    HIPCHK(hipStreamSynchronize(s->st));
    return OCN_OK;
}

int ocn_closure_detach(ocn_state* s) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    HIPCHK(hipStreamSynchronize(s->st));
    drop_graph(s);
    s->closure = false;
    s->kappa_conv = 0.0;
    s->ri_on = false;
    s->net = nullptr;
    s->d.kw = nullptr;
    s->d.kv = nullptr;
    s->kv_ws = nullptr;
    s->norm = nullptr; s->xb = s->h1b = s->h2b = nullptr; s->y = nullptr;
    s->din = s->h1 = s->h2 = s->dout = 0;
    return OCN_OK;
}

int ocn_closure_features(ocn_state* s, int32_t din, const float* norm_dev, float* x_dev) {
    if (!s || !x_dev) return fail(OCN_E_INVALID, "state and x must not be NULL");
    if (s->d.salinity) return fail(OCN_E_UNSUPPORTED, "the closure features take temperature-only states");
    if (din < 4 * s->g->nz + 3) return fail(OCN_E_INVALID, "din must be at least 4 nz + 3");
    if (ocn::features_lds(din) > 64 * 1024) return fail(OCN_E_UNSUPPORTED, "din too large");
    HIPCHK(s->esize == 4 ? ocn::launch_features<float>(s->d, din, norm_dev, x_dev, 0, s->st)
                         : ocn::launch_features<double>(s->d, din, norm_dev, x_dev, 0, s->st));
    return OCN_OK;
}

int ocn_closure_kappa(ocn_state* s, const float* y_dev, int32_t ldy) {
    if (!s || !y_dev) return fail(OCN_E_INVALID, "state and y must not be NULL");
    if (!s->closure) return fail(OCN_E_STATE, "no closure attached");
    if (ldy < s->g->nz) return fail(OCN_E_INVALID, "ldy must be at least nz");
    HIPCHK(s->esize == 4 ? ocn::launch_kappa_map<float>(s->d, y_dev, ldy, s->p.kappa, s->st)
                         : ocn::launch_kappa_map<double>(s->d, y_dev, ldy, s->p.kappa, s->st));
    return OCN_OK;
}

int ocn_stage_timing(ocn_state* s, int32_t enable) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    HIPCHK(hipStreamSynchronize(s->st));
    drop_events(s);
    s->timing = enable != 0;
    return OCN_OK;
}

int ocn_stage_times(ocn_state* s, double* ms, int32_t n, int64_t* steps) {
    if (!s || (!ms && n > 0) || n < 0) return fail(OCN_E_INVALID, "bad arguments");
    HIPCHK(hipStreamSynchronize(s->st));
    // events per step: closure | tendency | barotropic | column
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t b = 0; b + 4 < s->events.size(); b += 5)
        for (int q = 0; q < 4; ++q) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, s->events[b + q], s->events[b + q + 1]));
            acc[q] += t;
        }
    const double order[4] = {acc[1], acc[2], acc[3], acc[0]};  // tendency, barotropic, column, closure
    for (int q = 0; q < n && q < 4; ++q) ms[q] = order[q];
    if (steps) *steps = s->timed_steps;
    drop_events(s);
    return OCN_OK;
}

namespace {

// Copy the reduced values out and fill the diagnostics record.
int diag_finish(ocn_state* s, const double* dev_out, ocn_diag* out) {
    double r[ocn::DG_COUNT];
    HIPCHK(hipMemcpyAsync(r, dev_out, sizeof(r), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    out->step = s->step;
    out->time = s->time;
    out->tracer_content = r[ocn::DG_TRACER];
    out->volume = r[ocn::DG_VOLUME];
    out->volume_mean = r[ocn::DG_VOLUME_MEAN];
    out->kinetic_energy = r[ocn::DG_KE];
    out->wet_area = r[ocn::DG_WET_AREA];
    out->max_abs_u = r[ocn::DG_MAX_U];
    out->max_abs_v = r[ocn::DG_MAX_V];
    out->max_abs_w = r[ocn::DG_MAX_W];
    out->cfl_adv = r[ocn::DG_CFL];
    out->t_max = r[ocn::DG_T_MAX];
    out->t_min = -r[ocn::DG_NEG_T_MIN];
    out->eta_max = r[ocn::DG_ETA_MAX];
    out->eta_min = -r[ocn::DG_NEG_ETA_MIN];
    out->nonfinite = (int64_t)r[ocn::DG_NONFINITE];
    out->cfl_bt = s->cfl_bt;
    out->salt_content = r[ocn::DG_SALT];
    if (out->nonfinite > 0) return fail(OCN_E_UNSTABLE, "non-finite values in the state");
    return OCN_OK;
}

}  // namespace

int ocn_diagnostics(ocn_state* s, ocn_diag* out) {
    if (!s || !out) return fail(OCN_E_INVALID, "state and out must not be NULL");
    HIPCHK(s->esize == 4 ? ocn::launch_diagnostics<float>(s->d, s->st) : ocn::launch_diagnostics<double>(s->d, s->st));
    return diag_finish(s, s->d.diag_out, out);
}

int ocn_diagnostics_noalloc(ocn_state* s, ocn_diag* out) {
    if (!s || !out) return fail(OCN_E_INVALID, "state and out must not be NULL");
    int dev = 0;
    if (s->st) HIPCHK(hipStreamGetDevice(s->st, &dev));
    else HIPCHK(hipGetDevice(&dev));
    double* scratch = nullptr;
    int max_blocks = 0;
    HIPCHK(ocn::diag_scratch(dev, &scratch, &max_blocks));
    const long long blocks = (long long)((s->g->nx + 63) / 64) * ((s->g->ny + 3) / 4);
    if (blocks > max_blocks)
        return fail(OCN_E_UNSUPPORTED, "grid too large for the fixed diagnostics scratch: at most " +
                                           std::to_string((long long)max_blocks * 256) + " columns");
    DevState d = s->d;  // the same kernels, with the partials and results in the fixed scratch
    d.diag_part = scratch;
    d.diag_out = scratch + (size_t)max_blocks * ocn::DG_COUNT;
    d.diag_blocks = max_blocks;
    HIPCHK(s->esize == 4 ? ocn::launch_diagnostics<float>(d, s->st) : ocn::launch_diagnostics<double>(d, s->st));
    return diag_finish(s, d.diag_out, out);
}

namespace {

struct CkptHeader {
    uint64_t magic;
    int32_t version, esize, nx, ny, nz, h;
    int32_t first, t_set;
    int64_t step;
    double time;
};
constexpr uint64_t kCkptMagic = 0x4f434e434b505431ull;  // "OCNCKPT1"

// (device pointer, bytes) of every region a checkpoint carries, in order
std::vector<std::pair<void*, size_t>> ckpt_regions(ocn_state* s) {
    DevState& d = s->d;
    std::vector<std::pair<void*, size_t>> r;
    for (void* f : {d.u, d.v, d.t, d.gu, d.gv, d.gt}) r.push_back({base3(s, f), s->n3 * s->esize});
    if (d.salinity)
        for (void* f : {d.s, d.gs}) r.push_back({base3(s, f), s->n3 * s->esize});
    for (double* f : {d.eta, d.ubt, d.vbt, d.eta_mean, d.ubt_mean, d.vbt_mean, d.cu, d.cv})
        r.push_back({base2(s, f), s->n2 * sizeof(double)});
    return r;
}

size_t ckpt_size(ocn_state* s) {
    size_t n = sizeof(CkptHeader) + s->g->nz * sizeof(double) * (s->d.salinity ? 2 : 1);
    for (auto& r : ckpt_regions(s)) n += r.second;
    return n;
}

}  // namespace

int ocn_checkpoint_bytes(ocn_state* s, size_t* bytes) {
    if (!s || !bytes) return fail(OCN_E_INVALID, "state and bytes must not be NULL");
    *bytes = ckpt_size(s);
    return OCN_OK;
}

int ocn_checkpoint_save(ocn_state* s, void* host, size_t bytes) {
    if (!s || !host) return fail(OCN_E_INVALID, "state and host must not be NULL");
    if (bytes != ckpt_size(s)) return fail(OCN_E_INVALID, "buffer size differs from ocn_checkpoint_bytes");
    unsigned char* p = static_cast<unsigned char*>(host);
    CkptHeader h{kCkptMagic, 1, s->esize, s->g->nx, s->g->ny, s->g->nz, s->g->h, s->first, s->t_set ? 1 : 0,
                 s->step, s->time};
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    std::memcpy(p, s->tref.data(), s->g->nz * sizeof(double));
    p += s->g->nz * sizeof(double);
    if (s->d.salinity) {
        std::memcpy(p, s->sref.data(), s->g->nz * sizeof(double));
        p += s->g->nz * sizeof(double);
    }
    for (auto& r : ckpt_regions(s)) {
        HIPCHK(hipMemcpyAsync(p, r.first, r.second, hipMemcpyDeviceToHost, s->st));
        p += r.second;
    }
    HIPCHK(hipStreamSynchronize(s->st));
    return OCN_OK;
}

int ocn_checkpoint_load(ocn_state* s, const void* host, size_t bytes) {
    if (!s || !host) return fail(OCN_E_INVALID, "state and host must not be NULL");
    if (bytes != ckpt_size(s)) return fail(OCN_E_INVALID, "buffer size differs from ocn_checkpoint_bytes");
    const unsigned char* p = static_cast<const unsigned char*>(host);
    CkptHeader h;
    std::memcpy(&h, p, sizeof(h));
    if (h.magic != kCkptMagic || h.version != 1 || h.esize != s->esize || h.nx != s->g->nx || h.ny != s->g->ny ||
        h.nz != s->g->nz || h.h != s->g->h)
        return fail(OCN_E_INVALID, "checkpoint does not match this state's grid or precision");
    p += sizeof(h);
    std::vector<double> tref(s->g->nz), sref(s->g->nz, 0.0);
    std::memcpy(tref.data(), p, s->g->nz * sizeof(double));
    p += s->g->nz * sizeof(double);
    if (s->d.salinity) {
        std::memcpy(sref.data(), p, s->g->nz * sizeof(double));
        p += s->g->nz * sizeof(double);
    }
    for (auto& r : ckpt_regions(s)) {
        HIPCHK(hipMemcpyAsync(r.first, p, r.second, hipMemcpyHostToDevice, s->st));
        p += r.second;
    }
    HIPCHK(hipStreamSynchronize(s->st));
    s->tref = tref;
    if (s->d.salinity) {
        s->sref = sref;
        s->s_set = true;
    }
    s->t_set = h.t_set != 0;
    s->first = h.first;
    s->step = h.step;
    s->time = h.time;
    return s->esize == 4 ? upload_tables<float>(s) : upload_tables<double>(s);
}

int ocn_synchronize(ocn_state* s) {
    if (!s) return fail(OCN_E_INVALID, "state must not be NULL");
    HIPCHK(hipStreamSynchronize(s->st));
    return OCN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Ensembles

struct ocn_ensemble {
    std::vector<ocn_state*> members;
    ocn_params p{};
    hipStream_t st = nullptr;
    int esize = 8;
    int max_nz = 1;
    int first = 1;
    int tend_ty = 0;   // 0 = precision default
    int fuse = ocn::kBaroFuseDefault;
    DevState* d_members = nullptr;  // two tables of the members: as they are, and with
                                    // their tracer-history buffers swapped
    std::vector<DevState> tab[2];   // host copies of both tables
    int epar = 0;                   // the table the next step uses
    int4* d_tend = nullptr;
    int4* d_col = nullptr;
    int4* d_baro = nullptr;
    int* d_queue = nullptr;         // queue counters: 8 per launch of a step
    int persistent = 0;             // 1: persistent workgroups over per-XCD queues
    int n_tend = 0, n_col = 0, n_baro = 0;
    size_t cap_tend = 0;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
};

namespace {

struct EnsPlan {
    std::vector<size_t> member_off, member_bytes;
    size_t off_dev, off_tend, off_col, off_baro, off_queue, total;
    size_t cap_tend, cap_col, cap_baro;
};

size_t tend_tiles(const ocn_grid* g, int ty) {
    return (size_t)((g->nx + 62) / 63) * (size_t)((g->ny + ty - 2) / (ty - 1));
}

int ens_plan(const ocn_grid* const* grids, int n, const ocn_params* params, EnsPlan& P) {
    Layout L;
    P.cap_tend = P.cap_col = P.cap_baro = 0;
    for (int m = 0; m < n; ++m) {
        const size_t b = make_plan(grids[m], params->precision, params->n_substeps, params->salinity).total;
        P.member_off.push_back(L.add(b));
        P.member_bytes.push_back(b);
        P.cap_tend += tend_tiles(grids[m], 4);  // the larger of the two tile shapes
        P.cap_col += (size_t)((grids[m]->nx + 63) / 64) * grids[m]->ny;
        P.cap_baro += (size_t)((grids[m]->nx + ocn::kBaroTileX - 1) / ocn::kBaroTileX) *
                      ((grids[m]->ny + ocn::kBaroTileY - 1) / ocn::kBaroTileY);
    }
    P.off_dev = L.add(2 * (size_t)n * sizeof(DevState));
    P.off_tend = L.add(P.cap_tend * sizeof(int4));
    P.off_col = L.add(P.cap_col * sizeof(int4));
    P.off_baro = L.add(P.cap_baro * sizeof(int4));
    // tendency and column launches, and at most one barotropic launch per two substeps
    P.off_queue = L.add(8 * (size_t)(2 + ocn::baro_substeps(std::max(params->n_substeps, 1))) * sizeof(int));
    P.total = L.total;
    return OCN_OK;
}

// Host copy of the XCD dealing used by the single-state tendency kernel.
int xcd_slot(int b, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int x = b % 8, slot = b / 8;
    return (x < r) ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

int ens_tables(ocn_ensemble* e) {
    const int ty = ocn::tend_tile_rows(e->esize, e->tend_ty);
    std::vector<int4> logical;
    for (int m = 0; m < (int)e->members.size(); ++m) {
        const ocn_grid* g = e->members[m]->g;
        const int gx = (g->nx + 62) / 63, gy = (g->ny + ty - 2) / (ty - 1);
        for (int by = 0; by < gy; ++by)
            for (int bx = 0; bx < gx; ++bx) logical.push_back(make_int4(m, bx, by, 0));
    }
    const int nb = (int)logical.size();
    if ((size_t)nb > e->cap_tend) return fail(OCN_E_INVALID, "tile table overflow");
    std::vector<int4> hw(nb);
    for (int b = 0; b < nb; ++b) hw[b] = logical[xcd_slot(b, nb)];
    HIPCHK(hipMemcpyAsync(e->d_tend, hw.data(), nb * sizeof(int4), hipMemcpyHostToDevice, e->st));
    e->n_tend = nb;
    std::vector<int4> col, baro;
    for (int m = 0; m < (int)e->members.size(); ++m) {
        const ocn_grid* g = e->members[m]->g;
        for (int j = 0; j < g->ny; ++j)
            for (int bx = 0; bx < (g->nx + 63) / 64; ++bx) col.push_back(make_int4(m, bx, j, 0));
        for (int by = 0; by < (g->ny + ocn::kBaroTileY - 1) / ocn::kBaroTileY; ++by)
            for (int bx = 0; bx < (g->nx + ocn::kBaroTileX - 1) / ocn::kBaroTileX; ++bx)
                baro.push_back(make_int4(m, bx, by, 0));
    }
    // barotropic tiles dealt like the tendency's: each XCD a contiguous range
    std::vector<int4> baro_hw(baro.size());
    for (int b = 0; b < (int)baro.size(); ++b) baro_hw[b] = baro[xcd_slot(b, (int)baro.size())];
    HIPCHK(hipMemcpyAsync(e->d_col, col.data(), col.size() * sizeof(int4), hipMemcpyHostToDevice, e->st));
    HIPCHK(hipMemcpyAsync(e->d_baro, baro_hw.data(), baro_hw.size() * sizeof(int4), hipMemcpyHostToDevice, e->st));
    e->n_col = (int)col.size();
    e->n_baro = (int)baro.size();
    // member states with the ensemble's tile settings, and the same with the
    // tracer-history buffers swapped (the table of the step after)
    const size_t n = e->members.size();
    e->tab[0].clear();
    e->tab[1].clear();
    for (ocn_state* s : e->members) {
        s->d.tend_ty = e->tend_ty;
        s->d.baro_fuse = e->fuse;
        e->tab[0].push_back(s->d);
        DevState o = s->d;
        std::swap(o.gt, o.gt_out);
        std::swap(o.gs, o.gs_out);
        e->tab[1].push_back(o);
    }
    e->epar = 0;
    for (int q = 0; q < 2; ++q)
        HIPCHK(hipMemcpyAsync(e->d_members + q * n, e->tab[q].data(), n * sizeof(DevState), hipMemcpyHostToDevice,
                              e->st));
    HIPCHK(hipStreamSynchronize(e->st));
    return OCN_OK;
}

void drop_graph(ocn_ensemble* e) {
    for (int q = 0; q < 2; ++q) {
        if (e->exec[q]) (void)hipGraphExecDestroy(e->exec[q]);
        if (e->graph[q]) (void)hipGraphDestroy(e->graph[q]);
        e->exec[q] = nullptr;
        e->graph[q] = nullptr;
    }
}

int ens_enqueue(ocn_ensemble* e, int first) {
    const bool f32 = e->esize == 4;
    const int ty = ocn::tend_tile_rows(e->esize, e->tend_ty);
    const DevState* dm = e->d_members + (size_t)e->epar * e->members.size();
    int *qt = nullptr, *qc = nullptr, *qb = nullptr;
    if (e->persistent) {  // fresh counters for every launch of the step
        const int nq = 8 * (2 + ocn::baro_launches(e->p.n_substeps, e->fuse));
        HIPCHK(ocn::launch_zero_counters(e->d_queue, nq, e->st));
        qt = e->d_queue;
        qc = e->d_queue + 8;
        qb = e->d_queue + 16;
    }
    HIPCHK(f32 ? ocn::launch_tendency_batched<float>(dm, e->d_tend, e->n_tend, ty, first, qt, e->st)
               : ocn::launch_tendency_batched<double>(dm, e->d_tend, e->n_tend, ty, first, qt, e->st));
    HIPCHK(ocn::launch_barotropic_batched(dm, (int)e->members.size(), e->d_baro, e->n_baro, e->p.n_substeps, e->fuse,
                                          e->p.dt, qb, e->st));
    HIPCHK(f32 ? ocn::launch_column_batched<float>(dm, e->d_col, e->n_col, e->max_nz, qc, e->st)
               : ocn::launch_column_batched<double>(dm, e->d_col, e->n_col, e->max_nz, qc, e->st));
    return OCN_OK;
}

int ens_step(ocn_ensemble* e, int n) {
    int rc;
    for (int q = 0; q < n; ++q) {
        // a member stepped on its own since the tables were built has its
        // history buffers the other way round: rebuild the tables
        for (size_t m = 0; m < e->members.size(); ++m)
            if (e->members[m]->d.gt != e->tab[e->epar][m].gt) {
                if (e->st) HIPCHK(hipStreamSynchronize(e->st));
                drop_graph(e);
                if ((rc = ens_tables(e))) return rc;
                break;
            }
        if (e->first || !e->st) {
            if ((rc = ens_enqueue(e, e->first))) return rc;
        } else {
            const int par = e->epar;
            if (!e->exec[par]) {
                HIPCHK(hipStreamBeginCapture(e->st, hipStreamCaptureModeThreadLocal));
                rc = ens_enqueue(e, 0);
                hipGraph_t g = nullptr;
                hipError_t ce = hipStreamEndCapture(e->st, &g);
                if (rc) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc;
                }
                if (ce != hipSuccess) return fail(OCN_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
                e->graph[par] = g;
                HIPCHK(hipGraphInstantiate(&e->exec[par], e->graph[par], nullptr, nullptr, 0));
            }
            HIPCHK(hipGraphLaunch(e->exec[par], e->st));
        }
        e->first = 0;
        e->epar ^= 1;
        for (ocn_state* s : e->members) {
            s->first = 0;
            s->step += 1;
            s->time += s->p.dt;
            s->swap_history();
        }
    }
    return OCN_OK;
}

}  // namespace

int ocn_ensemble_arena_bytes(const ocn_grid* const* grids, int32_t n, const ocn_params* params, size_t* bytes) {
    if (!grids || n < 1 || !bytes) return fail(OCN_E_INVALID, "grids, n >= 1 and bytes are required");
    std::string why;
    if (!valid_params(params, why)) return fail(OCN_E_INVALID, why);
    for (int m = 0; m < n; ++m)
        if (!grids[m]) return fail(OCN_E_INVALID, "NULL grid");
    EnsPlan P;
    ens_plan(grids, n, params, P);
    *bytes = P.total;
    return OCN_OK;
}

int ocn_ensemble_init(const ocn_grid* const* grids, int32_t n, const ocn_params* params, void* device_arena,
                      size_t arena_bytes, void* hip_stream, ocn_ensemble** out) {
    try {
        if (!grids || n < 1 || !out || !device_arena) return fail(OCN_E_INVALID, "bad arguments");
        std::string why;
        if (!valid_params(params, why)) return fail(OCN_E_INVALID, why);
        if (reinterpret_cast<uintptr_t>(device_arena) % 256) return fail(OCN_E_INVALID, "arena must be 256-byte aligned");
        for (int m = 0; m < n; ++m)
            if (!grids[m]) return fail(OCN_E_INVALID, "NULL grid");
        if (params->salinity) return fail(OCN_E_UNSUPPORTED, "ensembles take temperature only");
        if (params->momentum_form) return fail(OCN_E_UNSUPPORTED, "ensembles take the flux form of momentum");
        EnsPlan P;
        ens_plan(grids, n, params, P);
        if (arena_bytes < P.total) return fail(OCN_E_NOMEM, "arena smaller than ocn_ensemble_arena_bytes");
        ocn_ensemble* e = new ocn_ensemble();
        e->p = *params;
        e->st = static_cast<hipStream_t>(hip_stream);
        e->esize = params->precision == OCN_FP32 ? 4 : 8;
        e->fuse = params->baro_fuse < 2 ? ocn::kBaroFuseDefault : params->baro_fuse;
        unsigned char* A = static_cast<unsigned char*>(device_arena);
        for (int m = 0; m < n; ++m) {
            ocn_state* s = nullptr;
            int rc = ocn_state_init(grids[m], params, A + P.member_off[m], P.member_bytes[m], hip_stream, &s);
            if (rc) {
                for (ocn_state* q : e->members) ocn_state_destroy(q);
                delete e;
                return rc;
            }
            e->members.push_back(s);
            e->max_nz = std::max(e->max_nz, grids[m]->nz);
        }
        e->d_members = reinterpret_cast<DevState*>(A + P.off_dev);
        e->d_tend = reinterpret_cast<int4*>(A + P.off_tend);
        e->d_col = reinterpret_cast<int4*>(A + P.off_col);
        e->d_baro = reinterpret_cast<int4*>(A + P.off_baro);
        e->d_queue = reinterpret_cast<int*>(A + P.off_queue);
        e->cap_tend = P.cap_tend;
        int rc = ens_tables(e);
        if (rc) {
            ocn_ensemble_destroy(e);
            return rc;
        }
        *out = e;
        return OCN_OK;
    } catch (const std::bad_alloc&) {
        return fail(OCN_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(OCN_E_INVALID, "unexpected error");
    }
}

void ocn_ensemble_destroy(ocn_ensemble* e) {
    if (!e) return;
    if (e->st) (void)hipStreamSynchronize(e->st);
    drop_graph(e);
    for (ocn_state* s : e->members) ocn_state_destroy(s);
    delete e;
}

int ocn_ensemble_member(ocn_ensemble* e, int32_t m, ocn_state** member) {
    if (!e || !member || m < 0 || m >= (int)e->members.size()) return fail(OCN_E_INVALID, "bad member index");
    *member = e->members[m];
    return OCN_OK;
}

int ocn_ensemble_step(ocn_ensemble* e, int32_t n) {
    if (!e) return fail(OCN_E_INVALID, "ensemble must not be NULL");
    if (n < 0) return fail(OCN_E_INVALID, "n must be >= 0");
    // a member set to forward Euler (for example after loading a checkpoint
    // taken at step 0) makes the next ensemble step a first step
    for (ocn_state* s : e->members)
        if (s->first) e->first = 1;
    return ens_step(e, n);
}

int ocn_ensemble_set_tiles(ocn_ensemble* e, int32_t tend_rows, int32_t baro_fuse, int32_t persistent) {
    if (!e) return fail(OCN_E_INVALID, "ensemble must not be NULL");
    if (!(tend_rows == 0 || tend_rows == 4 || tend_rows == 8)) return fail(OCN_E_INVALID, "tend_rows must be 0, 4 or 8");
    if (!(baro_fuse == 0 || (baro_fuse >= 2 && baro_fuse <= 8))) return fail(OCN_E_INVALID, "baro_fuse must be 0 or 2..8");
    if (persistent != 0 && persistent != 1) return fail(OCN_E_INVALID, "persistent must be 0 or 1");
    if (e->st) HIPCHK(hipStreamSynchronize(e->st));
    drop_graph(e);
    e->tend_ty = tend_rows;
    e->fuse = baro_fuse == 0 ? ocn::kBaroFuseDefault : baro_fuse;
    e->persistent = persistent;
    return ens_tables(e);
}

int ocn_ensemble_autotune(ocn_ensemble* e, int32_t trial_steps, int32_t* tend_rows, int32_t* baro_fuse,
                          int32_t* persistent, double* ms_per_step) {
    if (!e || trial_steps < 1) return fail(OCN_E_INVALID, "ensemble and trial_steps >= 1 are required");
    if (!e->st) return fail(OCN_E_UNSUPPORTED, "autotuning needs a non-default stream");
    // save every member so the trials leave the ensemble where it was
    std::vector<std::vector<unsigned char>> saved(e->members.size());
    for (size_t m = 0; m < e->members.size(); ++m) {
        size_t nb = 0;
        int rc = ocn_checkpoint_bytes(e->members[m], &nb);
        if (rc) return rc;
        saved[m].resize(nb);
        if ((rc = ocn_checkpoint_save(e->members[m], saved[m].data(), nb))) return rc;
    }
    const int first0 = e->first;
    const int rows_c[2] = {4, 8};
    const int fuse_c[4] = {5, 6, 7, 8};
    double best = 1e300;
    int brow = 0, bfuse = ocn::kBaroFuseDefault, bpers = 0;
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    int rc = OCN_OK;
    for (int p = 0; p < 2 && !rc; ++p) {
        for (int r : rows_c) {
            for (int f : fuse_c) {
                if ((rc = ocn_ensemble_set_tiles(e, r, f, p))) break;
                e->first = 0;
                if ((rc = ens_step(e, 1))) break;  // capture and warm up
                HIPCHK(hipEventRecord(a, e->st));
                if ((rc = ens_step(e, trial_steps))) break;
                HIPCHK(hipEventRecord(b, e->st));
                HIPCHK(hipEventSynchronize(b));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, a, b));
                const double per = ms / trial_steps;
                if (per < best) { best = per; brow = r; bfuse = f; bpers = p; }
            }
            if (rc) break;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    if ((rc = ocn_ensemble_set_tiles(e, brow, bfuse, bpers))) return rc;
    for (size_t m = 0; m < e->members.size(); ++m)
        if ((rc = ocn_checkpoint_load(e->members[m], saved[m].data(), saved[m].size()))) return rc;
    e->first = first0;
    for (ocn_state* s : e->members) s->first = first0;
    if (tend_rows) *tend_rows = brow;
    if (baro_fuse) *baro_fuse = bfuse;
    if (persistent) *persistent = bpers;
    if (ms_per_step) *ms_per_step = best;
    return OCN_OK;
}
