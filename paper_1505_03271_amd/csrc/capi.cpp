// C ABI of liblb (include/lb.h): handle lifecycle, grid metric, stepping,
// diagnostics.  No exception crosses the ABI; every entry point reports
// failures through its return code and lb_last_error().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lb.h"
#include "lb_kernels.h"

using namespace lbk;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(LB_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

size_t elem_size(int storage) {
    switch (storage) {
        case LB_F64: return 8;
        case LB_F32: return 4;
        default: return 2;
    }
}

bool is_split_storage(int storage) { return storage == LB_BF16S || storage == LB_F16S; }

// Bytes of one population state: 9 or 18 planes of populations, or the
// moment-split layout (FP32 moments + 16-bit residuals).
uint64_t state_size(int storage, bool thermal, uint64_t cells) {
    if (is_split_storage(storage)) return uint64_t(SplitLayout{thermal, int64_t(cells)}.bytes());
    return (thermal ? 18ull : 9ull) * cells * elem_size(storage);
}

// Centre of node k (ghosts included) on an axis with faces xi[0..n].
double node_pos(const std::vector<double>& xi, bool periodic, long k) {
    const long n = long(xi.size()) - 1;
    if (k >= 0 && k < n) return 0.5 * (xi[k] + xi[k + 1]);
    if (periodic) {
        const double L = xi[n] - xi[0];
        long m = k % n;
        if (m < 0) m += n;
        return 0.5 * (xi[m] + xi[m + 1]) + double((k - m) / n) * L;
    }
    if (k < 0) return 2.0 * xi[0] - node_pos(xi, periodic, -k - 1);
    return 2.0 * xi[n] - node_pos(xi, periodic, 2 * n - 1 - k);
}

// Lagrange weights at x of the parabola through nodes (a, b, c), in that order.
void lagrange3(double x, double a, double b, double c, double* w) {
    w[0] = (x - b) * (x - c) / ((a - b) * (a - c));
    w[1] = (x - a) * (x - c) / ((b - a) * (b - c));
    w[2] = (x - a) * (x - b) / ((c - a) * (c - b));
}

// QUICK face weights (sec. 2.2.3) for faces 0..n: 6 per face, laid out as
// documented in lb_kernels.h: up = (w_P, w_E, w_W) on nodes (k-1, k, k-2),
// dn = (w_E, w_P, w_EE) on nodes (k, k-1, k+1).
std::vector<double> quick_weights(const std::vector<double>& xi, bool periodic) {
    const long n = long(xi.size()) - 1;
    std::vector<double> out(size_t(n + 1) * 6);
    for (long k = 0; k <= n; ++k) {
        const double xf = xi[k];
        const double W = node_pos(xi, periodic, k - 2), P = node_pos(xi, periodic, k - 1);
        const double E = node_pos(xi, periodic, k), EE = node_pos(xi, periodic, k + 1);
        double w[3];
        lagrange3(xf, P, E, W, w);
        out[k * 6 + 0] = w[0];
        out[k * 6 + 1] = w[1];
        out[k * 6 + 2] = w[2];
        lagrange3(xf, E, P, EE, w);
        out[k * 6 + 3] = w[0];
        out[k * 6 + 4] = w[1];
        out[k * 6 + 5] = w[2];
    }
    return out;
}

// Four-point flux stencils of every cell of an axis (n cells, face weights fw
// from quick_weights): D * scale = sum coef * phi, with coef[0..3] on nodes
// i-2 .. i+1 for c = +1 and coef[4..7] on nodes i-1 .. i+2 for c = -1,
// scale = factor / width_i.  They combine the two faces of the cell:
//   c = +1:  D = ([phi]_{i+1/2} - [phi]_{i-1/2}) / dx_i
//   c = -1:  D = -([phi]_{i+1/2} - [phi]_{i-1/2}) / dx_i
std::vector<double> flux_stencils(const std::vector<double>& xi, const std::vector<double>& fw, double factor) {
    const size_t n = xi.size() - 1;
    std::vector<double> out(n * 8);
    for (size_t i = 0; i < n; ++i) {
        const double* L = &fw[i * 6];        // face i     (between i-1 and i)
        const double* Rr = &fw[(i + 1) * 6]; // face i + 1 (between i and i+1)
        const double sc = factor / (xi[i + 1] - xi[i]);
        // c = +1: face value up0 P + up1 E + up2 W
        out[i * 8 + 0] = sc * (-L[2]);
        out[i * 8 + 1] = sc * (Rr[2] - L[0]);
        out[i * 8 + 2] = sc * (Rr[0] - L[1]);
        out[i * 8 + 3] = sc * (Rr[1]);
        // c = -1: face value dn0 E + dn1 P + dn2 EE, flux sign -1
        out[i * 8 + 4] = sc * (L[4]);
        out[i * 8 + 5] = sc * (L[3] - Rr[4]);
        out[i * 8 + 6] = sc * (L[5] - Rr[3]);
        out[i * 8 + 7] = sc * (-Rr[5]);
    }
    return out;
}

// derivative at x0 of the parabola through (x0, x1, x2): weights of the values
void d_weights(double x0, double x1, double x2, double* w) {
    w[0] = 1.0 / (x0 - x1) + 1.0 / (x0 - x2);
    w[1] = (x0 - x2) / ((x1 - x0) * (x1 - x2));
    w[2] = (x0 - x1) / ((x2 - x0) * (x2 - x1));
}

}  // namespace

// kinds of timed launches: 0 FV predictor or single pass, 1 FV corrector,
// 2 ST, 3 FV fused step (predictor and corrector in one launch)
constexpr int TIMED_KINDS = 4;
// default interval of lb_set_rebase for split thermal storage
constexpr int64_t SPLIT_REBASE_EVERY = 100;

struct lb_sim {
    lb_params p{};
    int device = 0;   // the device current at lb_create
    int nsp = 1;
    int64_t plane = 0;
    size_t state_bytes = 0;
    hipStream_t stream = nullptr;
    void* A = nullptr;  // current state
    void* B = nullptr;  // predictor / next state
    int fused = -1;     // lb_set_fv_fused: 1 fused steps, 0 separate launches, -1 where they pay
    int chunk_f = 0;    // rows per work item of the fused step (0: chosen at its first launch)
    void* metric = nullptr;   // flux stencils: x pass0, y pass0, x pass1, y pass1 ([n][8] each)
    double* dxy = nullptr;    // dx[nx], dy[ny] in double
    double* partial = nullptr;
    double* dout = nullptr;
    float* tref = nullptr;    // per-row thermal reference of the stored g (thermal, non-F64 storage)
    float* qref = nullptr;    // per-row heat-flux reference of the g residuals (thermal, split storage)
    int64_t rebase_every = 0, since_rebase = 0;
    size_t metric_bytes = 0;
    bool has_grid = false, has_init = false, unstable = false;
    std::vector<double> xf, yf;
    int chunk_h = 0;
    int lanes = 0;            // FV item width: 0 chosen from nx, or FV_LANES / FV_NARROW
    int st_pairs = 1;         // ST, 16-bit storage: two cells per thread where nx is even
    lb_group* group = nullptr;  // the group this simulation is a member of, if any
    int group_slot = -1;
    // non-finite flag: raised by the kernels on the device (d_bad), copied to
    // pinned host memory (h_bad) after every lb_step
    int* d_bad = nullptr;
    int* h_bad = nullptr;
    // captured step graphs of STEP_GRAPH_STEPS steps, by the state they start
    // from (buffer A and steps since the last rebase) and the state they leave
    struct StepGraph {
        void* p0[2];        // A, B at the start
        int64_t since0;
        void* p1[2];        // and at the end
        int64_t since1;
        hipGraphExec_t exec;
    };
    std::vector<StepGraph> graphs;
    hipStream_t cap = nullptr;   // private stream the graphs are captured on (the handle's may be the null stream)
    // timing
    bool timing = false;
    std::vector<hipEvent_t> events;
    std::vector<int> kinds;  // kind of the launch that starts at event k
    size_t n_rec = 0;
    int64_t launches[TIMED_KINDS] = {};
    double ms[TIMED_KINDS] = {};
};

namespace {

int check_sim(const lb_sim* s) {
    if (!s) return fail(LB_EINVAL, "NULL handle");
    return LB_OK;
}

void group_forget(lb_sim* s);

// A group's captured launches hold the member's buffers and item layout, so
// a member is neither stepped nor changed except through its group.
int check_free(const lb_sim* s, const char* fn) {
    if (int rc = check_sim(s)) return rc;
    if (s->group) return fail(LB_ESTATE, "%s: the simulation is a group member (slot %d)", fn, s->group_slot);
    return LB_OK;
}

// Copy host arrays to new device buffers: all of them, or none (on failure
// the ones already made are freed and every *dst is left null).
struct Upload {
    void** dst;
    const void* src;
    size_t bytes;
};
int upload_all(std::initializer_list<Upload> ups, const char* fn) {
    hipError_t e = hipSuccess;
    for (const Upload& u : ups) {
        *u.dst = nullptr;
        if (e == hipSuccess) e = hipMalloc(u.dst, u.bytes);
        if (e == hipSuccess) e = hipMemcpy(*u.dst, u.src, u.bytes, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) return LB_OK;
    for (const Upload& u : ups)
        if (*u.dst) { (void)hipFree(*u.dst); *u.dst = nullptr; }
    return fail(e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE, "%s: %s", fn, hipGetErrorString(e));
}

// Drop the captured step graphs (their launches hold the handle's buffers,
// metric, launch shape and rebase schedule).
void drop_step_graphs(lb_sim* s) {
    for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
}

// Release every device allocation of a handle (safe on partial creation).
void release(lb_sim* s) {
    drop_step_graphs(s);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    s->cap = nullptr;
    if (s->d_bad) (void)hipFree(s->d_bad);
    if (s->h_bad) (void)hipHostFree(s->h_bad);
    s->d_bad = nullptr;
    s->h_bad = nullptr;
    if (s->A) (void)hipFree(s->A);
    if (s->B) (void)hipFree(s->B);
    if (s->metric) (void)hipFree(s->metric);
    if (s->dxy) (void)hipFree(s->dxy);
    if (s->partial) (void)hipFree(s->partial);
    if (s->dout) (void)hipFree(s->dout);
    if (s->tref) (void)hipFree(s->tref);
    if (s->qref) (void)hipFree(s->qref);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    s->events.clear();
}

// the buffer holding the current state: A, or for a member of a group that
// runs fused steps, whichever its phase names (waits for the group's work)
const void* member_state(const lb_sim* s);
bool in_fused_group(const lb_sim* s);

AuxArgs aux_args(const lb_sim* s) {
    AuxArgs a{};
    a.state = const_cast<void*>(member_state(s));
    a.nx = s->p.nx;
    a.ny = s->p.ny;
    a.plane = s->plane;
    a.thermal = s->p.thermal;
    const double dt = s->p.scheme == LB_ST ? 1.0 : s->p.dt;
    a.hdt = s->p.scheme == LB_FV_EULER ? 0.0 : 0.5 * dt;
    a.ax = s->p.ax;
    a.ay = s->p.ay;
    a.bg = s->p.thermal ? s->p.beta_g : 0.0;
    a.T0 = s->p.T0;
    a.ref_f = s->p.storage == LB_F64 ? 0.0 : s->p.rho_ref;
    a.ref_g = s->p.storage == LB_F64 ? 0.0 : s->p.T_ref;
    a.dx = s->dxy;
    a.dy = s->dxy + s->p.nx;
    a.grouped = s->p.scheme != LB_ST;
    a.tref = s->tref;
    a.qref = s->qref;
    return a;
}

template <class R>
void fill_stage_k(const lb_params& p, StageK<R>& k) {
    const double dt = p.dt;
    const bool f64 = p.storage == LB_F64;
    const double rf = f64 ? 0.0 : p.rho_ref, rg = f64 ? 0.0 : p.T_ref;
    double hdt, k1, kh, kc, kf, k1g, kcg;
    if (p.scheme == LB_FV_EULER) {
        hdt = 0; k1 = 0; kh = 0; kc = dt / p.tau; kf = dt; k1g = 0; kcg = dt / p.tau_g;
    } else {
        const double tt = p.tau + 0.5 * dt, ttg = p.tau_g + 0.5 * dt;
        hdt = 0.5 * dt; k1 = dt / (2.0 * tt); kh = 0.5 * dt; kc = dt / tt; kf = dt * (1.0 - dt / (2.0 * tt));
        k1g = dt / (2.0 * ttg); kcg = dt / ttg;
    }
    k.hdt = R(hdt);
    k.ax = R(p.ax);
    k.ay = R(p.ay);
    k.bg = R(p.thermal ? p.beta_g : 0.0);
    k.T0 = R(p.T0);
    k.ref_f = R(rf);
    k.ref_g = R(rg);
    k.k1 = R(k1); k.kh = R(kh); k.k1x3 = R(3 * k1); k.khx3 = R(3 * kh); k.omk1 = R(1 - k1);
    k.k1g = R(k1g); k.omk1g = R(1 - k1g);
    k.kc = R(kc); k.kf = R(kf); k.kcx3 = R(3 * kc); k.kfx3 = R(3 * kf); k.omkc = R(1 - kc); k.omkcg = R(1 - kcg);
    k.kcg = R(kcg);
    k.cP = R(kh - (1 - k1) * hdt);
    k.cB = R(kf - (1 - kc) * hdt);
}

// Narrow items (four FV_NARROW-lane items per block) unless the wide strips
// need fewer lanes for this width; narrow lanes are weighted 4% heavier (their
// halo share and exchange cost more per owned column).
bool narrow_strips(const lb_sim* s) {
    if (s->lanes) return s->lanes == FV_NARROW;
    const int64_t nx = s->p.nx;
    const int64_t wide = FV_LANES * ((nx + FV_LANES - 2 * FV_HALO - 1) / (FV_LANES - 2 * FV_HALO));
    const int64_t narrow = FV_NARROW * ((nx + FV_NARROW - 2 * FV_HALO - 1) / (FV_NARROW - 2 * FV_HALO));
    return narrow * 104 < wide * 100;
}
int strip_width(const lb_sim* s) { return (narrow_strips(s) ? FV_NARROW : FV_LANES) - 2 * FV_HALO; }

template <class R>
FvArgs<R> fv_args(const lb_sim* s, const void* src, void* dst, void* aux, bool corrector) {
    FvArgs<R> a{};
    a.src = src;
    a.dst = dst;
    a.aux = aux;
    const size_t es = elem_size(s->p.storage);
    a.state_bytes = uint32_t(s->state_bytes);
    a.group_bytes = uint32_t(4 * size_t(s->plane) * es);
    a.rest_off = uint32_t(8 * size_t(s->nsp) * size_t(s->plane) * es);
    a.nx = s->p.nx;
    a.ny = s->p.ny;
    a.wall_x = s->p.bc_x;   // LB_PERIODIC 0, LB_WALL 1, LB_DENSITY 2
    a.wall_y = s->p.bc_y;
    a.narrow = narrow_strips(s) ? 1 : 0;
    a.strip_w = strip_width(s);
    a.chunk_h = s->chunk_h;
    a.n_strips = (s->p.nx + a.strip_w - 1) / a.strip_w;
    a.n_items = a.n_strips * ((s->p.ny + a.chunk_h - 1) / a.chunk_h);
    const R* m = static_cast<const R*>(s->metric);
    const size_t nx8 = size_t(s->p.nx) * 8, ny8 = size_t(s->p.ny) * 8;
    const R* pass = m + (corrector ? nx8 + ny8 : 0);
    a.xcoef = pass;
    a.ycoef = pass + nx8;
    fill_stage_k<R>(s->p, a.k);
    a.Tb = R(s->p.T_bottom);
    a.Tt = R(s->p.T_top);
    a.rho_x0 = R(s->p.rho_x0);
    a.rho_x1 = R(s->p.rho_x1);
    a.tref = reinterpret_cast<const R*>(s->tref);  // float rows for FP32 arithmetic, NULL for FP64
    a.qref = reinterpret_cast<const R*>(s->qref);  // split storage only
    a.bad = s->d_bad;
    return a;
}

int record_event(lb_sim* s, int kind) {
    if (!s->timing) return LB_OK;
    if (s->n_rec == s->events.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        s->events.push_back(e);
        s->kinds.push_back(-1);
    }
    HIP_TRY(hipEventRecord(s->events[s->n_rec], s->stream));
    s->kinds[s->n_rec] = kind;
    ++s->n_rec;
    return LB_OK;
}

int fold_timing(lb_sim* s) {
    if (s->n_rec == 0) return LB_OK;
    HIP_TRY(hipEventSynchronize(s->events[s->n_rec - 1]));
    for (size_t k = 0; k + 1 < s->n_rec; ++k) {
        const int kind = s->kinds[k];
        if (kind < 0 || kind >= TIMED_KINDS) continue;
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, s->events[k], s->events[k + 1]));
        s->ms[kind] += t;
        s->launches[kind] += 1;
    }
    s->n_rec = 0;
    return LB_OK;
}

// Rows per FV work item: as tall as possible while every item of a launch
// is resident at once (one item per block), in steps of four rows.
int auto_chunk(const lb_sim* s) {
    const int n_strips = (s->p.nx + strip_width(s) - 1) / strip_width(s);
    int cap = fv_resident_blocks(s->p.storage, s->p.thermal, false);
    if (cap <= 0) cap = 512;
    if (narrow_strips(s)) cap *= 4;  // four items per block
    const int chunks = std::max(1, cap / n_strips);
    int h = (s->p.ny + chunks - 1) / chunks;
    h = ((h + 3) / 4) * 4;
    return std::max(4, h);   // small grids: short items, many of them (an item's march is serial)
}

int fv_launch(lb_sim* s, const void* src, void* dst, void* aux, bool corrector) {
    if (s->chunk_h <= 0) s->chunk_h = auto_chunk(s);
    int rc = record_event(s, corrector ? 1 : 0);
    if (rc) return rc;
    hipError_t e;
    if (s->p.storage == LB_F64) {
        FvArgs<double> a = fv_args<double>(s, src, dst, aux, corrector);
        e = launch_fv_pass(s->p.storage, s->p.thermal, corrector, &a, s->stream);
    } else {
        FvArgs<float> a = fv_args<float>(s, src, dst, aux, corrector);
        e = launch_fv_pass(s->p.storage, s->p.thermal, corrector, &a, s->stream);
    }
    if (e != hipSuccess) return fail(LB_EDEVICE, "FV kernel launch failed: %s", hipGetErrorString(e));
    return LB_OK;
}

// ---- fused steps (x periodic, semi-implicit + Heun) ----
// Fused steps: semi-implicit + Heun, periodic x, FP32 arithmetic (not FP64
// storage), wide strips (not forced narrow).
// The automatic setting uses them where they measured faster than separate
// launches on MI355X: every format and grid measured, 1024^2 to 4096^2, with
// and without g (with g: FP32 +21 to +99%, split 16-bit +10 to +23%, plain
// 16-bit +17 to +34%).
bool fused_pays(const lb_sim*) { return true; }
bool fused_eligible(const lb_sim* s) {
    return s->p.scheme == LB_FV_HEUN && s->p.bc_x == LB_PERIODIC && s->p.storage != LB_F64 &&
           s->lanes != FV_NARROW && (s->fused > 0 || (s->fused < 0 && fused_pays(s)));
}
int strip_width_fused(const lb_sim*) { return FV_LANES - 2 * FV_FUSED_HALO; }
int auto_chunk_fused(const lb_sim* s) {
    const int n_strips = (s->p.nx + strip_width_fused(s) - 1) / strip_width_fused(s);
    int cap = fv_fused_resident_blocks(s->p.storage, s->p.thermal);
    if (cap <= 0) cap = 256;
    const int chunks = std::max(1, cap / n_strips);
    int h = (s->p.ny + chunks - 1) / chunks;
    h = ((h + 3) / 4) * 4;
    return std::max(8, h);
}
template <class R>
FvArgs<R> fv_args_fused(const lb_sim* s, const void* cur, void* next) {
    FvArgs<R> a = fv_args<R>(s, cur, next, nullptr, false);            // the predictor's weights (dt)
    const FvArgs<R> c = fv_args<R>(s, cur, next, nullptr, true);
    a.xcoef2 = c.xcoef;                                                  // and the corrector's (dt/2)
    a.ycoef2 = c.ycoef;
    a.narrow = 0;
    a.strip_w = strip_width_fused(s);
    a.chunk_h = s->chunk_f;
    a.n_strips = (s->p.nx + a.strip_w - 1) / a.strip_w;
    a.n_items = a.n_strips * ((s->p.ny + a.chunk_h - 1) / a.chunk_h);
    return a;
}

// One fused step: f~n in cur, f~n+1 to next.
int fused_launch(lb_sim* s, const void* cur, void* next) {
    if (s->chunk_f <= 0) s->chunk_f = auto_chunk_fused(s);
    if (s->chunk_h <= 0) s->chunk_h = auto_chunk(s);   // fv_args' item count of the separate launches
    if (int rc = record_event(s, 3)) return rc;
    hipError_t e;
    if (s->p.storage == LB_F64) {
        FvArgs<double> a = fv_args_fused<double>(s, cur, next);
        e = launch_fv_fused(s->p.storage, s->p.thermal, &a, s->stream);
    } else {
        FvArgs<float> a = fv_args_fused<float>(s, cur, next);
        e = launch_fv_fused(s->p.storage, s->p.thermal, &a, s->stream);
    }
    if (e != hipSuccess) return fail(LB_EDEVICE, "FV fused kernel launch failed: %s", hipGetErrorString(e));
    return LB_OK;
}

int st_launch(lb_sim* s) {
    StArgs a{};
    a.src = s->A;
    a.dst = s->B;
    a.nx = s->p.nx;
    a.ny = s->p.ny;
    a.plane = s->plane;
    a.wall_x = s->p.bc_x == LB_WALL;
    a.wall_y = s->p.bc_y == LB_WALL;
    a.tau = s->p.tau;
    a.tau_g = s->p.tau_g;
    a.ax = s->p.ax;
    a.ay = s->p.ay;
    a.bg = s->p.thermal ? s->p.beta_g : 0.0;
    a.T0 = s->p.T0;
    a.T_bottom = s->p.T_bottom;
    a.T_top = s->p.T_top;
    a.ref_f = s->p.storage == LB_F64 ? 0.0 : s->p.rho_ref;
    a.ref_g = s->p.storage == LB_F64 ? 0.0 : s->p.T_ref;
    a.tref = s->tref;
    a.pairs = s->st_pairs;
    a.bad = s->d_bad;
    int rc = record_event(s, 2);
    if (rc) return rc;
    hipError_t e = launch_st(s->p.storage, s->p.thermal, (s->p.flags & LB_FLAG_STREAM_ONLY) != 0, a, s->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "ST kernel launch failed: %s", hipGetErrorString(e));
    std::swap(s->A, s->B);
    return LB_OK;
}

DiagArgs diag_args(const lb_sim* s) {
    DiagArgs d{};
    d.a = aux_args(s);
    const int ny = s->p.ny;
    const auto& yf = s->yf;
    const double H = yf[ny] - yf[0];
    const double dT = s->p.T_bottom - s->p.T_top;
    d.walls = s->p.thermal && s->p.bc_y == LB_WALL && dT != 0.0;
    if (d.walls) {
        const double y0 = 0.5 * (yf[0] + yf[1]), y1 = 0.5 * (yf[1] + yf[2]);
        const double z0 = 0.5 * (yf[ny - 1] + yf[ny]), z1 = 0.5 * (yf[ny - 2] + yf[ny - 1]);
        d_weights(yf[0], y0, y1, d.nub);
        d_weights(yf[ny], z0, z1, d.nut);
        d.nu_scale = -H / dT;
    }
    d.Tb = s->p.T_bottom;
    d.Tt = s->p.T_top;
    d.inv_Lx = 1.0 / (s->xf[s->p.nx] - s->xf[0]);
    return d;
}

int run_diagnostics(lb_sim* s, double* host8) {
    const DiagArgs d = diag_args(s);
    const int ny = s->p.ny;
    const double H = s->yf[ny] - s->yf[0];
    const double dT = s->p.T_bottom - s->p.T_top;
    hipError_t e = launch_diagnostics(s->p.storage, d, s->partial, s->dout, s->stream, DiagFinal{});
    if (e != hipSuccess) return fail(LB_EDEVICE, "diagnostics launch failed: %s", hipGetErrorString(e));
    double o[D_COUNT];
    HIP_TRY(hipMemcpyAsync(o, s->dout, sizeof o, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const double kappa = s->p.tau_g / 3.0;
    host8[0] = o[D_MASS];
    host8[1] = o[D_EKIN];
    host8[2] = o[D_ETH];
    host8[3] = d.walls ? o[D_NUB] : 0.0;
    host8[4] = d.walls ? o[D_NUT] : 0.0;
    host8[5] = d.walls ? 1.0 + H * (o[D_UT] / o[D_VOL]) / (kappa * dT) : 0.0;
    host8[6] = o[D_VOL];
    host8[7] = o[D_BAD];
    if (o[D_BAD] != 0.0) s->unstable = true;
    return LB_OK;
}

// Clear the non-finite flag (a new state).
int clear_flag(lb_sim* s) {
    HIP_TRY(hipMemsetAsync(s->d_bad, 0, sizeof(int), s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    *s->h_bad = 0;
    s->unstable = false;
    return LB_OK;
}

// Wait for the handle's stream and read its non-finite flag.
int poll_flag(lb_sim* s) {
    HIP_TRY(hipMemcpyAsync(s->h_bad, s->d_bad, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (*s->h_bad) s->unstable = true;
    return LB_OK;
}

bool flagged(lb_sim* s) {
    if (*static_cast<volatile int*>(s->h_bad)) s->unstable = true;
    return s->unstable;
}

// Enqueue n time steps as single launches (the stepping of lb_step).  With
// fused steps, a semi-implicit + Heun step is one launch from A to B, after
// which the two swap.
int enqueue_steps(lb_sim* s, int64_t nsteps) {
    const bool fused = s->p.scheme == LB_FV_HEUN && fused_eligible(s);
    int64_t n = 0;
    for (; n < nsteps; ++n) {
        int rc;
        switch (s->p.scheme) {
            case LB_FV_HEUN:
                if (fused) {
                    if ((rc = fused_launch(s, s->A, s->B))) return rc;               // f~n+1 -> B
                    std::swap(s->A, s->B);
                    break;
                }
                if ((rc = fv_launch(s, s->A, s->B, nullptr, false))) return rc;  // f~* -> B
                if ((rc = fv_launch(s, s->B, s->A, s->A, true))) return rc;      // reads f~n at its cell, f~n+1 -> A
                break;
            case LB_FV_SEMI:
            case LB_FV_EULER:
                if ((rc = fv_launch(s, s->A, s->B, nullptr, false))) return rc;
                std::swap(s->A, s->B);
                break;
            default:
                if ((rc = st_launch(s))) return rc;
        }
        if (s->tref && s->rebase_every > 0 && ++s->since_rebase >= s->rebase_every) {
            hipError_t e = launch_rebase(s->p.storage, aux_args(s), s->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "rebase launch failed: %s", hipGetErrorString(e));
            s->since_rebase = 0;
        }
    }
    return LB_OK;
}

// The captured graph of STEP_GRAPH_STEPS steps from the handle's current
// state (capturing it on first use).  Kernel arguments are captured by
// value, so a graph is valid while the buffers, metric, launch shape and
// rebase interval it was made with are unchanged; the calls that change
// them drop the graphs.
constexpr int64_t STEP_GRAPH_STEPS = 32;
constexpr size_t STEP_GRAPHS_KEPT = 8;
int step_graph(lb_sim* s, const lb_sim::StepGraph** out) {
    void** bufs[2] = {&s->A, &s->B};
    for (const auto& g : s->graphs) {
        bool same = g.since0 == s->since_rebase;
        for (int q = 0; q < 2; ++q) same = same && g.p0[q] == *bufs[q];
        if (same) { *out = &g; return LB_OK; }
    }
    // launch shapes that are chosen at the first launch, chosen before the capture
    if (s->p.scheme != LB_ST && s->chunk_h <= 0) s->chunk_h = auto_chunk(s);
    if (fused_eligible(s) && s->chunk_f <= 0) s->chunk_f = auto_chunk_fused(s);
    if (!s->cap) HIP_TRY(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));  // default priority
    lb_sim::StepGraph g{};
    for (int q = 0; q < 2; ++q) g.p0[q] = *bufs[q];
    g.since0 = s->since_rebase;
    hipStream_t user = s->stream;
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(s->cap, hipStreamCaptureModeRelaxed));
    s->stream = s->cap;   // the launches below are recorded, not run
    int rc = enqueue_steps(s, STEP_GRAPH_STEPS);
    s->stream = user;
    hipError_t e = hipStreamEndCapture(s->cap, &graph);
    for (int q = 0; q < 2; ++q) {
        g.p1[q] = *bufs[q];
        *bufs[q] = g.p0[q];   // the graph has not run yet
    }
    g.since1 = s->since_rebase;
    s->since_rebase = g.since0;
    if (rc != LB_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc != LB_OK ? rc : fail(LB_EDEVICE, "lb_step: graph capture failed: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step: graph instantiation failed: %s", hipGetErrorString(e));
    if (s->graphs.size() >= STEP_GRAPHS_KEPT) {
        (void)hipGraphExecDestroy(s->graphs.front().exec);
        s->graphs.erase(s->graphs.begin());
    }
    s->graphs.push_back(g);
    *out = &s->graphs.back();
    return LB_OK;
}

}  // namespace

// ---- diagnostics without allocation (lb_diagnostics_noalloc) ------------
// Its partial sums live in this file-scope device array: one copy per GPU,
// held until the process ends, shared by every call on that GPU.  Host code
// never uses the array's name as an address: it takes the address that
// hipGetSymbolAddress returns with the device current (looked up once per
// device, on the first call there).
constexpr int NOALLOC_PARTIALS = DIAG_BLOCKS * D_COUNT;
constexpr int NOALLOC_DEVICES = 64;
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

namespace {

std::mutex g_scratch_mu;
double* g_scratch[NOALLOC_DEVICES] = {};

// Address of this device's scratch array (dev must be the current device).
int scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= NOALLOC_DEVICES) return fail(LB_EINVAL, "device %d: at most %d devices", dev, NOALLOC_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LB_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch[dev];
    return LB_OK;
}

template <class T>
int upload_temp(const T* host, size_t n, T** dev, hipStream_t st) {
    HIP_TRY(hipMalloc(dev, n * sizeof(T)));
    hipError_t e = hipMemcpyAsync(*dev, host, n * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        return fail(LB_EDEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    return LB_OK;
}

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

int lb_stream_probe(size_t bytes, void* stream, double* out) {
    if (!out) return fail(LB_EINVAL, "lb_stream_probe: out is NULL");
    const size_t n = bytes / 16;
    if (n < (size_t(16) << 20) / 16) return fail(LB_EINVAL, "lb_stream_probe: need at least 16 MiB per buffer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *a = nullptr, *b = nullptr, *d = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (d) (void)hipFree(d);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e = hipMalloc(&a, n * 16);
    if (e == hipSuccess) e = hipMalloc(&b, n * 16);
    if (e == hipSuccess) e = hipMalloc(&d, n * 16);
    if (e != hipSuccess) {
        release();
        return fail(LB_ENOMEM, "lb_stream_probe: %s", hipGetErrorString(e));
    }
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, n * 16, st);
    if (e == hipSuccess) e = hipMemsetAsync(b, 0, n * 16, st);
    if (e == hipSuccess) e = hipMemsetAsync(d, 0, n * 16, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // best of three launch shapes (4, 8 and 16 blocks of 256 lanes per CU)
    const int grids[] = {1024, 2048, 4096};
    const double moved[] = {2.0, 3.0, 2.0};  // buffers of n * 16 bytes moved per sweep
    const int reps = 10;
    for (int kind = 0; kind < 3 && e == hipSuccess; ++kind) {
        double best = 0.0;
        for (int g : grids) {
            for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch_stream(kind, g, a, b, d, n, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_stream(kind, g, a, b, d, n, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms > 0.f) best = std::max(best, moved[kind] * double(n) * 16.0 * reps / (double(ms) * 1e6));
        }
        out[kind] = best;
    }
    release();
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_stream_probe: %s", hipGetErrorString(e));
    return LB_OK;
}

int lb_grid_uniform(int64_t n, double L, double* faces) {
    if (n < 1 || !faces || !(L > 0)) return fail(LB_EINVAL, "lb_grid_uniform: bad arguments");
    for (int64_t i = 0; i <= n; ++i) faces[i] = L * double(i) / double(n);
    return LB_OK;
}

int lb_grid_tanh(int64_t n, double L, double stretch, double* faces) {
    if (n < 1 || !faces || !(L > 0) || !(stretch > 0)) return fail(LB_EINVAL, "lb_grid_tanh: bad arguments");
    // xi_i = L/2 (1 + tanh((2i/n - 1) atanh(s1)) / s1) with s1 = tanh(stretch)
    const double s1 = std::tanh(stretch);
    for (int64_t i = 0; i <= n; ++i)
        faces[i] = 0.5 * L * (1.0 + std::tanh((2.0 * double(i) / double(n) - 1.0) * stretch) / s1);
    faces[0] = 0.0;
    faces[n] = L;
    return LB_OK;
}

int lb_grid_sinh(int64_t n, double L, double s2, double* faces) {
    if (n < 2 || (n & 1) || !faces || !(L > 0) || !(s2 > 0))
        return fail(LB_EINVAL, "lb_grid_sinh: needs even n >= 2, L > 0, s2 > 0");
    // eq:grids: A sinh(s2 i / n) up to the middle face, mirrored above it
    const double A = 0.5 * L / std::sinh(0.5 * s2);
    for (int64_t i = 0; i <= n; ++i)
        faces[i] = 2 * i <= n ? A * std::sinh(s2 * double(i) / double(n)) : L - A * std::sinh(s2 * double(n - i) / double(n));
    faces[0] = 0.0;
    faces[n] = L;
    return LB_OK;
}

int lb_grid_chebyshev(int64_t n, double L, double* faces) {
    if (n < 1 || !faces || !(L > 0)) return fail(LB_EINVAL, "lb_grid_chebyshev: bad arguments");
    const double pi = 3.14159265358979323846;
    for (int64_t i = 0; i <= n; ++i) faces[i] = 0.5 * L * (1.0 - std::cos(pi * double(i) / double(n)));
    faces[0] = 0.0;
    faces[n] = L;
    return LB_OK;
}

int lb_create(const lb_params* p, lb_sim** out) {
    try {
        if (!p || !out) return fail(LB_EINVAL, "lb_create: NULL argument");
        *out = nullptr;
        if (p->nx < 4 || p->ny < 4) return fail(LB_EINVAL, "lb_create: nx and ny must be >= 4 (got %d, %d)", p->nx, p->ny);
        if (p->scheme < LB_FV_HEUN || p->scheme > LB_ST) return fail(LB_EINVAL, "lb_create: unknown scheme %d", p->scheme);
        if (p->storage < LB_F64 || p->storage > LB_F16S) return fail(LB_EINVAL, "lb_create: unknown storage %d", p->storage);
        if (is_split_storage(p->storage) && p->scheme == LB_ST)
            return fail(LB_EINVAL, "lb_create: moment-split storage (LB_BF16S, LB_F16S) is for the FV schemes only");
        if (!(p->tau > 0) || (p->thermal && !(p->tau_g > 0))) return fail(LB_EINVAL, "lb_create: tau and tau_g must be > 0");
        if (p->scheme != LB_ST && !(p->dt > 0)) return fail(LB_EINVAL, "lb_create: dt must be > 0");
        if ((p->bc_x != LB_PERIODIC && p->bc_x != LB_WALL && p->bc_x != LB_DENSITY) ||
            (p->bc_y != LB_PERIODIC && p->bc_y != LB_WALL))
            return fail(LB_EINVAL, "lb_create: bad boundary kind (fixed density is available on x only)");
        if (p->bc_x == LB_DENSITY && (p->scheme == LB_ST || p->thermal))
            return fail(LB_EINVAL, "lb_create: fixed-density boundaries are for the flow populations of the FV schemes");
        if (p->bc_x == LB_DENSITY && !(p->rho_x0 > 0 && p->rho_x1 > 0))
            return fail(LB_EINVAL, "lb_create: fixed densities rho_x0, rho_x1 must be > 0");
        if ((p->flags & LB_FLAG_STREAM_ONLY) && p->scheme != LB_ST)
            return fail(LB_EINVAL, "lb_create: LB_FLAG_STREAM_ONLY needs LB_ST");
        if (state_size(p->storage, p->thermal != 0, uint64_t(p->nx) * uint64_t(p->ny)) >= (1ull << 32))
            return fail(LB_EINVAL, "lb_create: the population state must be smaller than 4 GiB (nx*ny too large for this storage)");
        lb_sim* s = new (std::nothrow) lb_sim();
        if (!s) return fail(LB_ENOMEM, "lb_create: out of host memory");
        s->p = *p;
        if (s->p.scheme == LB_ST) s->p.dt = 1.0;
        s->nsp = p->thermal ? 2 : 1;
        s->fused = -1;   // fused steps where they pay (fused_pays)
        // Split thermal storage renews its references every 100 steps by
        // default: its 16-bit g residuals otherwise also carry the mean
        // vertical heat flux, and small departures from it (a convection roll
        // growing out of the conductive state) round away.
        s->rebase_every = p->thermal && is_split_storage(p->storage) ? SPLIT_REBASE_EVERY : 0;

        s->plane = int64_t(p->nx) * p->ny;
        s->state_bytes = size_t(state_size(p->storage, p->thermal != 0, uint64_t(s->plane)));
        s->stream = static_cast<hipStream_t>(p->stream);
        s->chunk_h = 0;  // chosen at the first FV launch from the occupancy
        hipError_t e = hipGetDevice(&s->device);
        if (e != hipSuccess) {
            delete s;
            return fail(LB_EDEVICE, "lb_create: no device: %s", hipGetErrorString(e));
        }
        if ((e = hipMalloc(&s->A, s->state_bytes)) != hipSuccess || (e = hipMalloc(&s->B, s->state_bytes)) != hipSuccess ||
            (e = hipMalloc(&s->partial, sizeof(double) * DIAG_BLOCKS * D_COUNT)) != hipSuccess ||
            (e = hipMalloc(&s->dout, sizeof(double) * D_COUNT)) != hipSuccess ||
            (p->thermal && p->storage != LB_F64 && (e = hipMalloc(&s->tref, sizeof(float) * p->ny)) != hipSuccess) ||
            (p->thermal && is_split_storage(p->storage) && (e = hipMalloc(&s->qref, sizeof(float) * p->ny)) != hipSuccess) ||
            (e = hipMalloc(&s->d_bad, sizeof(int))) != hipSuccess ||
            (e = hipHostMalloc(&s->h_bad, sizeof(int), hipHostMallocDefault)) != hipSuccess ||
            (e = hipMemset(s->d_bad, 0, sizeof(int))) != hipSuccess) {
            release(s);
            delete s;
            return fail(e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE, "lb_create: device allocation failed: %s",
                        hipGetErrorString(e));
        }
        *s->h_bad = 0;
        *out = s;
        return LB_OK;
    } catch (...) {
        return fail(LB_ENOMEM, "lb_create: unexpected failure");
    }
}

void lb_destroy(lb_sim* s) {
    if (!s) return;
    if (s->group && lb_group_remove(s->group, s->group_slot) != LB_OK) group_forget(s);
    (void)hipStreamSynchronize(s->stream);
    release(s);
    delete s;
}

int lb_set_grid(lb_sim* s, const double* x_faces, int64_t n_xf, const double* y_faces, int64_t n_yf) {
    if (int rc = check_free(s, "lb_set_grid")) return rc;
    try {
        if (!x_faces || !y_faces) return fail(LB_EINVAL, "lb_set_grid: NULL faces");
        if (n_xf != s->p.nx + 1 || n_yf != s->p.ny + 1)
            return fail(LB_EINVAL, "lb_set_grid: need nx+1 = %d and ny+1 = %d faces", s->p.nx + 1, s->p.ny + 1);
        for (int64_t i = 0; i + 1 < n_xf; ++i)
            if (!(x_faces[i + 1] > x_faces[i])) return fail(LB_EINVAL, "lb_set_grid: x faces not increasing at %lld", (long long)i);
        for (int64_t i = 0; i + 1 < n_yf; ++i)
            if (!(y_faces[i + 1] > y_faces[i])) return fail(LB_EINVAL, "lb_set_grid: y faces not increasing at %lld", (long long)i);
        if (s->p.scheme == LB_ST) {
            for (int64_t i = 0; i < n_xf; ++i)
                if (std::fabs(x_faces[i] - x_faces[0] - double(i)) > 1e-12) return fail(LB_EINVAL, "lb_set_grid: ST needs unit spacing in x");
            for (int64_t i = 0; i < n_yf; ++i)
                if (std::fabs(y_faces[i] - y_faces[0] - double(i)) > 1e-12) return fail(LB_EINVAL, "lb_set_grid: ST needs unit spacing in y");
        }
        std::vector<double> xf(x_faces, x_faces + n_xf), yf(y_faces, y_faces + n_yf);
        const int nx = s->p.nx, ny = s->p.ny;
        std::vector<double> xw = quick_weights(xf, s->p.bc_x == LB_PERIODIC);
        std::vector<double> yw = quick_weights(yf, s->p.bc_y == LB_PERIODIC);
        // pass 0: predictor / single pass (factor dt); pass 1: Heun corrector (dt/2)
        std::vector<double> m;
        for (double factor : {s->p.dt, 0.5 * s->p.dt}) {
            std::vector<double> a = flux_stencils(xf, xw, factor), b = flux_stencils(yf, yw, factor);
            m.insert(m.end(), a.begin(), a.end());
            m.insert(m.end(), b.begin(), b.end());
        }
        std::vector<double> dxy(size_t(nx) + ny);
        for (int i = 0; i < nx; ++i) dxy[i] = xf[i + 1] - xf[i];
        for (int j = 0; j < ny; ++j) dxy[nx + j] = yf[j + 1] - yf[j];
        std::vector<float> mf;
        if (s->p.storage != LB_F64) mf.assign(m.begin(), m.end());
        const void* mh = s->p.storage == LB_F64 ? static_cast<const void*>(m.data()) : mf.data();
        const size_t mbytes = s->p.storage == LB_F64 ? m.size() * sizeof(double) : mf.size() * sizeof(float);
        // the new grid goes to new buffers; the old one stays in use if this fails
        void* metric = nullptr;
        void* dxy_d = nullptr;
        if (int rc = upload_all({{&metric, mh, mbytes}, {&dxy_d, dxy.data(), dxy.size() * sizeof(double)}}, "lb_set_grid"))
            return rc;
        if (hipError_t e = hipStreamSynchronize(s->stream); e != hipSuccess) {
            (void)hipFree(metric);
            (void)hipFree(dxy_d);
            return fail(LB_EDEVICE, "set_grid: %s", hipGetErrorString(e));
        }
        drop_step_graphs(s);
        if (s->metric) (void)hipFree(s->metric);
        if (s->dxy) (void)hipFree(s->dxy);
        s->metric = metric;
        s->dxy = static_cast<double*>(dxy_d);
        s->metric_bytes = mbytes;
        s->xf.swap(xf);
        s->yf.swap(yf);
        s->has_grid = true;
        return LB_OK;
    } catch (...) {
        return fail(LB_ENOMEM, "lb_set_grid: out of host memory");
    }
}

int lb_init(lb_sim* s, const double* rho, const double* ux, const double* uy, const double* T) {
    if (int rc = check_free(s, "lb_init")) return rc;
    if (!s->has_grid) return fail(LB_ESTATE, "lb_init: call lb_set_grid first");
    if (!rho || !ux || !uy || (s->p.thermal && !T)) return fail(LB_EINVAL, "lb_init: NULL field");
    const size_t n = size_t(s->plane);
    if (s->tref) {
        // the stored g are offsets from w_a times the row mean of the initial T
        std::vector<float> tr(s->p.ny);
        for (int j = 0; j < s->p.ny; ++j) {
            double m = 0.0;
            for (int i = 0; i < s->p.nx; ++i) m += T[size_t(j) * s->p.nx + i];
            tr[j] = float(m / s->p.nx);
        }
        HIP_TRY(hipMemcpy(s->tref, tr.data(), sizeof(float) * tr.size(), hipMemcpyHostToDevice));
    }
    if (s->qref) {
        // the equilibrium start has no heat flux in its residuals
        std::vector<float> z(s->p.ny, 0.0f);
        HIP_TRY(hipMemcpy(s->qref, z.data(), sizeof(float) * z.size(), hipMemcpyHostToDevice));
    }
    double *d[4] = {nullptr, nullptr, nullptr, nullptr};
    const double* h[4] = {rho, ux, uy, s->p.thermal ? T : rho};
    int rc = LB_OK;
    for (int q = 0; q < 4 && rc == LB_OK; ++q) rc = upload_temp(h[q], n, &d[q], s->stream);
    if (rc == LB_OK) {
        AuxArgs a = aux_args(s);
        hipError_t e = launch_init(s->p.storage, a, d[0], d[1], d[2], d[3], s->stream);
        if (e != hipSuccess) rc = fail(LB_EDEVICE, "init launch failed: %s", hipGetErrorString(e));
        else if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) rc = fail(LB_EDEVICE, "init failed: %s", hipGetErrorString(e));
    }
    for (double* p : d) if (p) (void)hipFree(p);
    if (rc == LB_OK) rc = clear_flag(s);
    if (rc == LB_OK) s->has_init = true;
    return rc;
}

int lb_step(lb_sim* s, int64_t nsteps) {
    if (int rc = check_free(s, "lb_step")) return rc;
    if (!s->has_init) return fail(LB_ESTATE, "lb_step: call lb_init (or lb_set_state) first");
    if (nsteps < 0) return fail(LB_EINVAL, "lb_step: negative step count");
    if (flagged(s)) return fail(LB_EUNSTABLE, "lb_step: non-finite populations were detected");
    if (nsteps == 0) return LB_OK;
    // Whole blocks of STEP_GRAPH_STEPS steps replay a captured graph, unless
    // every launch is timed or the caller is capturing the stream itself.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s->stream, &cap));
    const bool graphs = !s->timing && cap == hipStreamCaptureStatusNone;
    int64_t left = nsteps;
    while (graphs && left >= STEP_GRAPH_STEPS) {
        const lb_sim::StepGraph* g = nullptr;
        if (int rc = step_graph(s, &g)) return rc;
        HIP_TRY(hipGraphLaunch(g->exec, s->stream));
        s->A = g->p1[0];
        s->B = g->p1[1];
        s->since_rebase = g->since1;
        left -= STEP_GRAPH_STEPS;
    }
    if (int rc = enqueue_steps(s, left)) return rc;
    if (int rc = record_event(s, -1)) return rc;
    // the flag as of the end of these steps, read by the next call
    HIP_TRY(hipMemcpyAsync(s->h_bad, s->d_bad, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    return LB_OK;
}

int lb_sync(lb_sim* s) {
    if (int rc = check_sim(s)) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (flagged(s)) return fail(LB_EUNSTABLE, "lb_sync: non-finite populations were detected");
    return LB_OK;
}

int lb_moments(lb_sim* s, double* rho, double* ux, double* uy, double* T) {
    if (int rc = check_sim(s)) return rc;
    if (!s->has_init) return fail(LB_ESTATE, "lb_moments: no state");
    const size_t n = size_t(s->plane);
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, 4 * n * sizeof(double)));
    AuxArgs a = aux_args(s);
    hipError_t e = launch_moments(s->p.storage, a, d, d + n, d + 2 * n, d + 3 * n, s->stream);
    double* h[4] = {rho, ux, uy, T};
    for (int q = 0; q < 4 && e == hipSuccess; ++q)
        if (h[q]) e = hipMemcpyAsync(h[q], d + q * n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_moments failed: %s", hipGetErrorString(e));
    return LB_OK;
}

int lb_diagnostics(lb_sim* s, double* out) {
    if (int rc = check_sim(s)) return rc;
    if (!out) return fail(LB_EINVAL, "lb_diagnostics: NULL output");
    if (!s->has_init) return fail(LB_ESTATE, "lb_diagnostics: no state");
    if (int rc = run_diagnostics(s, out)) return rc;
    return poll_flag(s);
}

int lb_diagnostics_noalloc(lb_sim* s, double* out_device) {
    if (int rc = check_sim(s)) return rc;
    if (!out_device) return fail(LB_EINVAL, "lb_diagnostics_noalloc: NULL output");
    if (!s->has_init) return fail(LB_ESTATE, "lb_diagnostics_noalloc: no state");
    if (in_fused_group(s))   // which buffer holds its state is known on the device only
        return fail(LB_ESTATE, "lb_diagnostics_noalloc: a member of a group that runs fused steps");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != s->device)
        return fail(LB_EINVAL, "lb_diagnostics_noalloc: device %d is current, the handle is on device %d", dev, s->device);
    const int64_t need = int64_t(diag_blocks(s->plane)) * D_COUNT;
    if (need > NOALLOC_PARTIALS)
        return fail(LB_EINVAL, "lb_diagnostics_noalloc: %lld partial sums needed, the scratch holds %d",
                    (long long)need, NOALLOC_PARTIALS);
    double* partial = nullptr;
    if (int rc = scratch_address(dev, &partial)) return rc;
    const DiagArgs d = diag_args(s);
    DiagFinal fin{};
    fin.finish = 1;
    fin.walls = d.walls;
    fin.H = s->yf[s->p.ny] - s->yf[0];
    fin.kappa = s->p.tau_g / 3.0;
    fin.dT = s->p.T_bottom - s->p.T_top;
    hipError_t e = launch_diagnostics(s->p.storage, d, partial, out_device, s->stream, fin);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_diagnostics_noalloc: launch failed: %s", hipGetErrorString(e));
    return LB_OK;
}

int lb_profiles(lb_sim* s, double* out, int64_t n_out) {
    if (int rc = check_sim(s)) return rc;
    const int ny = s->p.ny;
    if (!s->p.thermal) return fail(LB_EINVAL, "lb_profiles: needs a thermal run");
    if (!out || n_out != 6 * int64_t(ny)) return fail(LB_EINVAL, "lb_profiles: need an output of 6 * ny = %lld doubles", (long long)(6 * int64_t(ny)));
    if (!s->has_init) return fail(LB_ESTATE, "lb_profiles: no state");
    try {
        double* d = nullptr;
        HIP_TRY(hipMalloc(&d, sizeof(double) * PROFILE_ROWS * ny));
        hipError_t e = launch_profiles(s->p.storage, aux_args(s), 1.0 / (s->xf[s->p.nx] - s->xf[0]), d, s->stream);
        std::vector<double> h(size_t(PROFILE_ROWS) * ny);
        if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        (void)hipFree(d);
        if (e != hipSuccess) return fail(LB_EDEVICE, "lb_profiles: %s", hipGetErrorString(e));
        const double* Tm = h.data();
        for (int j = 0; j < ny; ++j) {
            out[j] = Tm[j];
            out[ny + j] = std::sqrt(std::max(0.0, h[size_t(ny) + j] - Tm[j] * Tm[j]));
            out[2 * ny + j] = std::sqrt(h[2 * size_t(ny) + j]);
            out[3 * ny + j] = std::sqrt(h[3 * size_t(ny) + j]);
            out[4 * ny + j] = h[4 * size_t(ny) + j];
            out[5 * ny + j] = 0.0;
        }
        const double dT = s->p.T_bottom - s->p.T_top;
        if (s->p.bc_y == LB_WALL && dT != 0.0 && ny >= 2) {
            const auto& yf = s->yf;
            const double H = yf[ny] - yf[0], kappa = s->p.tau_g / 3.0;
            auto yc = [&](int j) { return 0.5 * (yf[j] + yf[j + 1]); };
            for (int j = 0; j < ny; ++j) {
                // derivative at y_j of the parabola through three (position, value) points
                double x0, x1, x2, v0, v1, v2;
                if (j == 0) { x0 = yf[0]; v0 = s->p.T_bottom; x1 = yc(0); v1 = Tm[0]; x2 = yc(1); v2 = Tm[1]; }
                else if (j == ny - 1) { x0 = yc(ny - 2); v0 = Tm[ny - 2]; x1 = yc(ny - 1); v1 = Tm[ny - 1]; x2 = yf[ny]; v2 = s->p.T_top; }
                else { x0 = yc(j - 1); v0 = Tm[j - 1]; x1 = yc(j); v1 = Tm[j]; x2 = yc(j + 1); v2 = Tm[j + 1]; }
                const double y = yc(j);
                const double dTdy = v0 * (2 * y - x1 - x2) / ((x0 - x1) * (x0 - x2)) +
                                    v1 * (2 * y - x0 - x2) / ((x1 - x0) * (x1 - x2)) +
                                    v2 * (2 * y - x0 - x1) / ((x2 - x0) * (x2 - x1));
                out[5 * ny + j] = (h[4 * size_t(ny) + j] - kappa * dTdy) / (kappa * dT / H);
            }
        }
        return LB_OK;
    } catch (...) {
        return fail(LB_ENOMEM, "lb_profiles: out of host memory");
    }
}

int lb_nusselt(lb_sim* s, double* nu_bottom, double* nu_top, double* nu_vol) {
    if (int rc = check_sim(s)) return rc;
    if (!s->p.thermal || s->p.bc_y != LB_WALL || s->p.T_bottom == s->p.T_top)
        return fail(LB_EINVAL, "lb_nusselt: needs a thermal run with y walls at different temperatures");
    if (!s->has_init) return fail(LB_ESTATE, "lb_nusselt: no state");
    double o[8];
    if (int rc = run_diagnostics(s, o)) return rc;
    if (int rc = poll_flag(s)) return rc;
    if (nu_bottom) *nu_bottom = o[3];
    if (nu_top) *nu_top = o[4];
    if (nu_vol) *nu_vol = o[5];
    if (s->unstable) return fail(LB_EUNSTABLE, "lb_nusselt: the simulation holds non-finite populations");
    return LB_OK;
}

int lb_get_populations(lb_sim* s, double* f, double* g) {
    if (int rc = check_sim(s)) return rc;
    if (!f) return fail(LB_EINVAL, "lb_get_populations: NULL f");
    if (!s->has_init) return fail(LB_ESTATE, "lb_get_populations: no state");
    const size_t n = size_t(s->nsp) * 9 * size_t(s->plane);
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, n * sizeof(double)));
    hipError_t e = launch_get_pops(s->p.storage, aux_args(s), d, s->stream);
    const size_t nf = 9 * size_t(s->plane);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, nf * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && s->p.thermal && g) e = hipMemcpyAsync(g, d + nf, nf * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_get_populations failed: %s", hipGetErrorString(e));
    return LB_OK;
}

int lb_set_populations(lb_sim* s, const double* f, const double* g) {
    if (int rc = check_free(s, "lb_set_populations")) return rc;
    if (!f || (s->p.thermal && !g)) return fail(LB_EINVAL, "lb_set_populations: NULL input");
    if (!s->has_grid) return fail(LB_ESTATE, "lb_set_populations: call lb_set_grid first");
    const size_t nf = 9 * size_t(s->plane);
    try {
        // the per-row references the state is encoded with, as lb_init sets
        // them: the row means of T = sum g, and no heat-flux reference
        if (s->tref) {
            std::vector<float> tr(s->p.ny);
            for (int j = 0; j < s->p.ny; ++j) {
                double m = 0.0;
                for (int i = 0; i < s->p.nx; ++i)
                    for (int a = 0; a < 9; ++a) m += g[size_t(a) * size_t(s->plane) + size_t(j) * s->p.nx + i];
                tr[j] = float(m / s->p.nx);
            }
            HIP_TRY(hipMemcpy(s->tref, tr.data(), sizeof(float) * tr.size(), hipMemcpyHostToDevice));
        }
        if (s->qref) {
            std::vector<float> z(s->p.ny, 0.0f);
            HIP_TRY(hipMemcpy(s->qref, z.data(), sizeof(float) * z.size(), hipMemcpyHostToDevice));
        }
    } catch (...) {
        return fail(LB_ENOMEM, "lb_set_populations: out of host memory");
    }
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, size_t(s->nsp) * nf * sizeof(double)));
    hipError_t e = hipMemcpyAsync(d, f, nf * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && s->p.thermal) e = hipMemcpyAsync(d + nf, g, nf * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = launch_set_pops(s->p.storage, aux_args(s), d, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_set_populations failed: %s", hipGetErrorString(e));
    if (int rc = clear_flag(s)) return rc;
    s->since_rebase = 0;
    s->has_init = true;
    return LB_OK;
}

// The checkpoint blob: the population state, then the per-row references
// (thermal, T_ref; split, the heat-flux reference) the state is encoded with.
size_t ref_bytes(const lb_sim* s) {
    return (s->tref ? sizeof(float) * size_t(s->p.ny) : 0) + (s->qref ? sizeof(float) * size_t(s->p.ny) : 0);
}

size_t lb_state_bytes(const lb_sim* s) { return s ? s->state_bytes + ref_bytes(s) : 0; }

int lb_get_state(lb_sim* s, void* host, size_t bytes) {
    if (int rc = check_sim(s)) return rc;
    const size_t need = s->state_bytes + ref_bytes(s);
    if (!host || bytes != need) return fail(LB_EINVAL, "lb_get_state: need %zu bytes", need);
    if (!s->has_init) return fail(LB_ESTATE, "lb_get_state: no state");
    char* h = static_cast<char*>(host);
    const size_t row = sizeof(float) * size_t(s->p.ny);
    HIP_TRY(hipMemcpyAsync(h, member_state(s), s->state_bytes, hipMemcpyDeviceToHost, s->stream));
    h += s->state_bytes;
    if (s->tref) { HIP_TRY(hipMemcpyAsync(h, s->tref, row, hipMemcpyDeviceToHost, s->stream)); h += row; }
    if (s->qref) HIP_TRY(hipMemcpyAsync(h, s->qref, row, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return LB_OK;
}

int lb_set_state(lb_sim* s, const void* host, size_t bytes) {
    if (int rc = check_free(s, "lb_set_state")) return rc;
    const size_t need = s->state_bytes + ref_bytes(s);
    if (!host || bytes != need) return fail(LB_EINVAL, "lb_set_state: need %zu bytes", need);
    if (!s->has_grid) return fail(LB_ESTATE, "lb_set_state: call lb_set_grid first");
    const char* h = static_cast<const char*>(host);
    const size_t row = sizeof(float) * size_t(s->p.ny);
    HIP_TRY(hipMemcpyAsync(s->A, h, s->state_bytes, hipMemcpyHostToDevice, s->stream));
    h += s->state_bytes;
    if (s->tref) { HIP_TRY(hipMemcpyAsync(s->tref, h, row, hipMemcpyHostToDevice, s->stream)); h += row; }
    if (s->qref) HIP_TRY(hipMemcpyAsync(s->qref, h, row, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (int rc = clear_flag(s)) return rc;
    s->has_init = true;
    return LB_OK;
}

int lb_set_timing(lb_sim* s, int enable) {
    if (int rc = check_sim(s)) return rc;
    if (s->timing && !enable) {
        if (int rc = fold_timing(s)) return rc;
    }
    s->timing = enable != 0;
    for (int k = 0; k < TIMED_KINDS; ++k) { s->launches[k] = 0; s->ms[k] = 0; }
    s->n_rec = 0;
    return LB_OK;
}

int lb_kernel_times(lb_sim* s, int64_t* launches, double* total_ms) {
    if (int rc = check_sim(s)) return rc;
    if (!launches || !total_ms) return fail(LB_EINVAL, "lb_kernel_times: NULL output");
    if (int rc = fold_timing(s)) return rc;
    for (int k = 0; k < TIMED_KINDS; ++k) { launches[k] = s->launches[k]; total_ms[k] = s->ms[k]; }
    return LB_OK;
}

size_t lb_device_bytes(const lb_sim* s) {
    if (!s) return 0;
    return 2 * s->state_bytes + s->metric_bytes + (s->tref ? sizeof(float) * size_t(s->p.ny) : 0) + (s->qref ? sizeof(float) * size_t(s->p.ny) : 0) + sizeof(double) * (size_t(s->p.nx) + s->p.ny) +
           sizeof(double) * (DIAG_BLOCKS * D_COUNT + D_COUNT);
}

int lb_rebase(lb_sim* s) {
    if (int rc = check_free(s, "lb_rebase")) return rc;
    if (!s->has_init) return fail(LB_ESTATE, "lb_rebase: no state");
    if (!s->tref) return LB_OK;
    hipError_t e = launch_rebase(s->p.storage, aux_args(s), s->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "rebase launch failed: %s", hipGetErrorString(e));
    s->since_rebase = 0;
    return LB_OK;
}

int lb_set_rebase(lb_sim* s, int64_t every) {
    if (int rc = check_free(s, "lb_set_rebase")) return rc;
    if (every < 0) return fail(LB_EINVAL, "lb_set_rebase: negative interval");
    s->rebase_every = every;
    s->since_rebase = 0;
    drop_step_graphs(s);
    return LB_OK;
}

int lb_set_st_pairs(lb_sim* s, int on) {
    if (int rc = check_sim(s)) return rc;
    if (on != 0 && on != 1) return fail(LB_EINVAL, "lb_set_st_pairs: on must be 0 or 1");
    s->st_pairs = on;
    drop_step_graphs(s);
    return LB_OK;
}

int lb_set_fv_lanes(lb_sim* s, int lanes) {
    if (int rc = check_free(s, "lb_set_fv_lanes")) return rc;
    if (lanes != 0 && lanes != FV_LANES && lanes != FV_NARROW)
        return fail(LB_EINVAL, "lb_set_fv_lanes: lanes must be 0, %d or %d", FV_NARROW, FV_LANES);
    s->lanes = lanes;
    s->chunk_h = 0;  // re-chosen at the next step for the new item width
    s->chunk_f = 0;
    drop_step_graphs(s);
    return LB_OK;
}

int lb_set_fv_chunk(lb_sim* s, int rows) {
    if (int rc = check_free(s, "lb_set_fv_chunk")) return rc;
    if (rows < 1) return fail(LB_EINVAL, "lb_set_fv_chunk: rows must be >= 1");
    s->chunk_h = rows;
    s->chunk_f = std::max(rows, 2);   // a fused item holds at least two rows
    drop_step_graphs(s);
    return LB_OK;
}

int lb_get_fv_fused(const lb_sim* s, int* on) {
    if (!s || !on) return fail(LB_EINVAL, "lb_get_fv_fused: NULL argument");
    *on = s->fused;
    return LB_OK;
}

int lb_set_fv_fused(lb_sim* s, int on) {
    if (int rc = check_free(s, "lb_set_fv_fused")) return rc;
    if (on < -1 || on > 1) return fail(LB_EINVAL, "lb_set_fv_fused: on must be -1, 0 or 1");
    s->fused = on;
    drop_step_graphs(s);
    return LB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- groups --

struct lb_group {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int max_sims = 0;
    std::vector<lb_sim*> sims;  // slot -> member (nullptr if free)
    int storage = -1, thermal = -1;
    // fused steps (every member eligible): per slot two argument blocks of
    // the fused step, one per direction of the member's pair of buffers, and
    // the phase that says which holds its state (flipped by the tick kernel;
    // settled into the member's A and B at every rebuild and removal)
    bool fused = false;
    void* d_fargs = nullptr;
    int* d_phase = nullptr;
    void* d_args = nullptr;     // 2 FvArgs per slot (separate launches: predictor, corrector)
    int2* d_items = nullptr;
    size_t items_cap = 0;
    int n_items = 0;            // all items; the first n_wide are wide-strip items
    int n_wide = 0;
    int64_t* d_left = nullptr;
    // renewal of the members' thermal references (lb_set_rebase), per slot:
    // interval (0: never), steps since the last renewal, due after this step
    int64_t* d_every = nullptr;
    int64_t* d_since = nullptr;
    int* d_due = nullptr;
    void* d_aux = nullptr;      // 2 AuxArgs per slot (the state in the member's A, in its B)
    int2* d_ritems = nullptr;   // (slot, row) of the members that renew their references
    size_t ritems_cap = 0;
    int n_ritems = 0;
    int chunk = 0;              // rows per work item: 0 chosen at each rebuild (group_chunk), else fixed
    std::vector<int> stale;     // free slots whose remaining-steps counter is to be cleared at the next rebuild
    bool dirty = true;
    hipGraphExec_t exec = nullptr;
    int64_t exec_steps = 0;
};

namespace {

// Drop a member from its group's slot table without touching the device
// (its destruction after a failed lb_group_remove): the group's next step
// rebuilds its launches without it.
void group_forget(lb_sim* s) {
    lb_group* g = s->group;
    g->sims[s->group_slot] = nullptr;
    g->stale.push_back(s->group_slot);
    g->dirty = true;
    s->group = nullptr;
    s->group_slot = -1;
    bool any = false;
    for (lb_sim* m : g->sims) any = any || m;
    if (!any) { g->storage = -1; g->thermal = -1; }
}

// Rows per work item for the current members.  All items of one launch have
// the same height h, so with B(h) blocks and `cap` of them resident at once
// a launch takes about ceil(B / cap) rounds of h + extra row times (an item
// also marches rows before and after its chunk and sets up its rings: 3 for
// the separate passes, 6 for a fused step, whose first half marches four
// rows more).  Pick the h of 16..512 (steps of 8) with the least such time:
// tall items when the members fill the chip many times over, short ones
// when few members are left.
int group_chunk(const lb_group* g, bool fused) {
    int cap = fused ? fv_fused_resident_blocks(g->storage, g->thermal != 0)
                    : fv_resident_blocks(g->storage, g->thermal != 0, false);
    if (cap <= 0) cap = fused ? 256 : 512;
    const int extra = fused ? 6 : 3;
    int best_h = 64;
    int64_t best_t = INT64_MAX;
    for (int h = 16; h <= 512; h += 8) {
        int64_t wide = 0, narrow = 0;
        for (const lb_sim* s : g->sims) {
            if (!s) continue;
            const int sw = fused ? strip_width_fused(s) : strip_width(s);
            const int64_t n = int64_t((s->p.nx + sw - 1) / sw) * ((s->p.ny + h - 1) / h);
            (!fused && narrow_strips(s) ? narrow : wide) += n;
        }
        const int64_t blocks = wide + (narrow + 3) / 4;
        const int64_t t = ((blocks + cap - 1) / cap) * (h + extra);
        if (t <= best_t) { best_t = t; best_h = h; }
    }
    return best_h;
}

bool in_fused_group(const lb_sim* s) { return s->group && s->group->fused; }

const void* member_state(const lb_sim* s) {
    const lb_group* g = s->group;
    if (!g || !g->fused) return s->A;
    int ph = 0;
    if (hipStreamSynchronize(g->stream) != hipSuccess ||
        hipMemcpy(&ph, g->d_phase + s->group_slot, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return s->A;
    return ph ? s->B : s->A;
}

// Settle the members' phases of fused group steps into their host state
// pointers (a member whose state is in its B swaps A and B) and clear them,
// so that every member's state is in its A again.
int group_settle(lb_group* g) {
    if (!g->fused) return LB_OK;
    HIP_TRY(hipStreamSynchronize(g->stream));
    std::vector<int> ph(size_t(g->max_sims), 0);
    HIP_TRY(hipMemcpy(ph.data(), g->d_phase, sizeof(int) * g->max_sims, hipMemcpyDeviceToHost));
    for (int k = 0; k < g->max_sims; ++k)
        if (g->sims[k] && ph[k]) std::swap(g->sims[k]->A, g->sims[k]->B);
    std::fill(ph.begin(), ph.end(), 0);
    HIP_TRY(hipMemcpy(g->d_phase, ph.data(), sizeof(int) * g->max_sims, hipMemcpyHostToDevice));
    return LB_OK;
}

void group_drop_graph(lb_group* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    g->exec = nullptr;
    g->exec_steps = 0;
}

template <class R>
void group_fill_args(lb_group* g, std::vector<char>& host) {
    for (int k = 0; k < g->max_sims; ++k) {
        lb_sim* s = g->sims[k];
        if (!s) continue;
        FvArgs<R> pa, ca;
        if (g->fused) {   // state in A: A -> B; state in B: B -> A
            pa = fv_args_fused<R>(s, s->A, s->B);
            ca = fv_args_fused<R>(s, s->B, s->A);
        } else {
            pa = fv_args<R>(s, s->A, s->B, nullptr, false);
            ca = fv_args<R>(s, s->B, s->A, s->A, true);
        }
        std::memcpy(&host[(2 * size_t(k)) * sizeof(FvArgs<R>)], &pa, sizeof pa);
        std::memcpy(&host[(2 * size_t(k) + 1) * sizeof(FvArgs<R>)], &ca, sizeof ca);
    }
}

int group_rebuild(lb_group* g) {
    if (int rc = group_settle(g)) return rc;
    // fused steps when every member can take them (otherwise separate passes)
    bool fused = g->storage >= 0;
    for (const lb_sim* s : g->sims)
        if (s) fused = fused && fused_eligible(s);
    g->fused = fused;
    if (g->storage >= 0) {
        int h = g->chunk > 0 ? g->chunk : group_chunk(g, fused);
        if (fused) h = std::max(h, 2);   // a fused item holds at least two rows
        for (lb_sim* s : g->sims)
            if (s) s->chunk_h = s->chunk_f = h;
    }
    const size_t ab = fv_args_bytes(g->storage);
    std::vector<char> host(2 * size_t(g->max_sims) * ab, 0);
    if (g->storage == LB_F64) group_fill_args<double>(g, host);
    else group_fill_args<float>(g, host);
    // fused: every member's items (wide strips); otherwise the items of
    // wide-strip members first, then those of narrow-strip ones
    std::vector<int2> items;
    int n_wide = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < g->max_sims; ++k) {
            lb_sim* s = g->sims[k];
            if (!s || (!fused && narrow_strips(s) != (pass == 1)) || (fused && pass == 1)) continue;
            const int sw = fused ? strip_width_fused(s) : strip_width(s);
            const int n = ((s->p.nx + sw - 1) / sw) * ((s->p.ny + s->chunk_h - 1) / s->chunk_h);
            for (int q = 0; q < n; ++q) items.push_back(int2{k, q});
            if (pass == 0) n_wide += n;
        }
    HIP_TRY(hipStreamSynchronize(g->stream));
    HIP_TRY(hipMemcpy(fused ? g->d_fargs : g->d_args, host.data(), host.size(), hipMemcpyHostToDevice));
    for (int k : g->stale) {
        const int64_t zero = 0;
        if (!g->sims[k]) HIP_TRY(hipMemcpy(g->d_left + k, &zero, sizeof zero, hipMemcpyHostToDevice));
    }
    g->stale.clear();
    if (items.size() > g->items_cap) {
        if (g->d_items) (void)hipFree(g->d_items);
        g->d_items = nullptr;
        g->items_cap = std::max<size_t>(items.size(), 2 * g->items_cap);
        HIP_TRY(hipMalloc(&g->d_items, g->items_cap * sizeof(int2)));
    }
    if (!items.empty()) HIP_TRY(hipMemcpy(g->d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
    g->n_items = int(items.size());
    g->n_wide = n_wide;
    // the rows renewed by the members with a rebase interval, and their
    // arguments (the state in A, and in B after an odd number of fused steps)
    std::vector<int2> ritems;
    std::vector<AuxArgs> aux(2 * size_t(g->max_sims));
    std::vector<int64_t> every(size_t(g->max_sims), 0);
    for (int k = 0; k < g->max_sims; ++k) {
        lb_sim* s = g->sims[k];
        if (!s || !s->tref || s->rebase_every <= 0) continue;
        aux[2 * k] = aux[2 * k + 1] = aux_args(s);
        if (fused) aux[2 * k + 1].state = s->B;
        every[k] = s->rebase_every;
        for (int j = 0; j < s->p.ny; ++j) ritems.push_back(int2{k, j});
    }
    HIP_TRY(hipMemcpy(g->d_aux, aux.data(), aux.size() * sizeof(AuxArgs), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->d_every, every.data(), every.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    if (ritems.size() > g->ritems_cap) {
        if (g->d_ritems) (void)hipFree(g->d_ritems);
        g->d_ritems = nullptr;
        g->ritems_cap = std::max<size_t>(ritems.size(), 2 * g->ritems_cap);
        HIP_TRY(hipMalloc(&g->d_ritems, g->ritems_cap * sizeof(int2)));
    }
    if (!ritems.empty())
        HIP_TRY(hipMemcpy(g->d_ritems, ritems.data(), ritems.size() * sizeof(int2), hipMemcpyHostToDevice));
    g->n_ritems = int(ritems.size());
    group_drop_graph(g);
    g->dirty = false;
    return LB_OK;
}

// Enqueue nsteps group steps on the group's stream (one fused step, or one
// predictor and one corrector, then one counter tick per step).
hipError_t group_enqueue(lb_group* g, int64_t nsteps) {
    int* phase = g->fused ? g->d_phase : nullptr;
    for (int64_t n = 0; n < nsteps; ++n) {
        const int nw = g->n_wide, nn = g->n_items - g->n_wide;
        hipError_t e;
        if (g->fused) {
            e = launch_fv_fused_multi(g->storage, g->thermal, g->d_fargs, g->d_items, g->n_items, g->d_left, phase,
                                      g->stream);
        } else {
            e = launch_fv_multi(g->storage, g->thermal, false, g->d_args, g->d_items, nw, nn, g->d_left, g->stream);
            if (e == hipSuccess)
                e = launch_fv_multi(g->storage, g->thermal, true, g->d_args, g->d_items, nw, nn, g->d_left, g->stream);
        }
        if (e == hipSuccess) e = launch_tick(g->d_left, g->max_sims, g->d_every, g->d_since, g->d_due, phase, g->stream);
        if (e == hipSuccess && g->n_ritems > 0)
            e = launch_rebase_multi(g->storage, static_cast<const AuxArgs*>(g->d_aux), g->d_ritems, g->n_ritems,
                                    g->d_due, phase, g->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int lb_group_create(int32_t max_sims, void* stream, lb_group** out) {
    if (!out || max_sims < 1 || max_sims > 65536) return fail(LB_EINVAL, "lb_group_create: 1 <= max_sims <= 65536");
    *out = nullptr;
    lb_group* g = new (std::nothrow) lb_group();
    if (!g) return fail(LB_ENOMEM, "lb_group_create: out of host memory");
    g->max_sims = max_sims;
    g->sims.assign(max_sims, nullptr);
    hipError_t e = hipSuccess;
    if (stream) {
        g->stream = static_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);  // default priority
        g->own_stream = e == hipSuccess;
    }
    const size_t ab = std::max(fv_args_bytes(LB_F64), fv_args_bytes(LB_F32));
    if (e == hipSuccess) e = hipMalloc(&g->d_args, 2 * size_t(max_sims) * ab);
    if (e == hipSuccess) e = hipMalloc(&g->d_fargs, 2 * size_t(max_sims) * ab);
    if (e == hipSuccess) e = hipMalloc(&g->d_phase, sizeof(int) * max_sims);
    if (e == hipSuccess) e = hipMalloc(&g->d_left, sizeof(int64_t) * max_sims);
    if (e == hipSuccess) e = hipMalloc(&g->d_every, sizeof(int64_t) * max_sims);
    if (e == hipSuccess) e = hipMalloc(&g->d_since, sizeof(int64_t) * max_sims);
    if (e == hipSuccess) e = hipMalloc(&g->d_due, sizeof(int) * max_sims);
    if (e == hipSuccess) e = hipMalloc(&g->d_aux, 2 * sizeof(AuxArgs) * max_sims);
    if (e == hipSuccess) {
        std::vector<int64_t> z(max_sims, 0);
        e = hipMemcpy(g->d_left, z.data(), sizeof(int64_t) * max_sims, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(g->d_phase, z.data(), sizeof(int) * max_sims, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(g->d_every, z.data(), sizeof(int64_t) * max_sims, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(g->d_since, z.data(), sizeof(int64_t) * max_sims, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        lb_group_destroy(g);
        return fail(LB_EDEVICE, "lb_group_create: %s", hipGetErrorString(e));
    }
    *out = g;
    return LB_OK;
}

void lb_group_destroy(lb_group* g) {
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->d_phase) (void)group_settle(g);   // the members keep their latest state in A
    for (lb_sim* m : g->sims)
        if (m) { m->group = nullptr; m->group_slot = -1; m->chunk_h = m->chunk_f = 0; }
    group_drop_graph(g);
    if (g->d_args) (void)hipFree(g->d_args);
    if (g->d_fargs) (void)hipFree(g->d_fargs);
    if (g->d_phase) (void)hipFree(g->d_phase);
    if (g->d_items) (void)hipFree(g->d_items);
    if (g->d_left) (void)hipFree(g->d_left);
    if (g->d_every) (void)hipFree(g->d_every);
    if (g->d_since) (void)hipFree(g->d_since);
    if (g->d_due) (void)hipFree(g->d_due);
    if (g->d_aux) (void)hipFree(g->d_aux);
    if (g->d_ritems) (void)hipFree(g->d_ritems);
    if (g->own_stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

int lb_group_add(lb_group* g, lb_sim* s, int64_t steps, int32_t* slot) {
    if (!g || !s || !slot) return fail(LB_EINVAL, "lb_group_add: NULL argument");
    if (steps < 0) return fail(LB_EINVAL, "lb_group_add: negative step count");
    if (s->p.scheme != LB_FV_HEUN) return fail(LB_EINVAL, "lb_group_add: members must use LB_FV_HEUN");
    if (!s->has_init) return fail(LB_ESTATE, "lb_group_add: the simulation has no state yet");
    if (g->storage >= 0 && (s->p.storage != g->storage || s->p.thermal != g->thermal))
        return fail(LB_EINVAL, "lb_group_add: members must share storage format and thermal flag");
    if (s->group == g) return fail(LB_EINVAL, "lb_group_add: already a member");
    if (s->group) return fail(LB_ESTATE, "lb_group_add: already a member of another group");
    int k = 0;
    while (k < g->max_sims && g->sims[k]) ++k;
    if (k == g->max_sims) return fail(LB_ENOMEM, "lb_group_add: all %d slots are taken", g->max_sims);
    HIP_TRY(hipStreamSynchronize(g->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const int zero = 0;
    HIP_TRY(hipMemcpy(g->d_left + k, &steps, sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->d_since + k, &s->since_rebase, sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->d_phase + k, &zero, sizeof(int), hipMemcpyHostToDevice));   // its state is in its A
    g->storage = s->p.storage;
    g->thermal = s->p.thermal;
    g->sims[k] = s;
    s->group = g;
    s->group_slot = k;
    drop_step_graphs(s);   // the group sets its own item height
    g->dirty = true;
    *slot = k;
    return LB_OK;
}

int lb_group_remove(lb_group* g, int32_t slot) {
    if (!g || slot < 0 || slot >= g->max_sims || !g->sims[slot]) return fail(LB_EINVAL, "lb_group_remove: bad slot");
    HIP_TRY(hipStreamSynchronize(g->stream));
    const int64_t zero = 0;
    HIP_TRY(hipMemcpy(g->d_left + slot, &zero, sizeof zero, hipMemcpyHostToDevice));
    lb_sim* s = g->sims[slot];
    HIP_TRY(hipMemcpy(&s->since_rebase, g->d_since + slot, sizeof(int64_t), hipMemcpyDeviceToHost));
    if (g->fused) {   // after an odd number of fused steps its state is in its B
        int ph = 0;
        HIP_TRY(hipMemcpy(&ph, g->d_phase + slot, sizeof(int), hipMemcpyDeviceToHost));
        if (ph) std::swap(s->A, s->B);
        const int zero = 0;
        HIP_TRY(hipMemcpy(g->d_phase + slot, &zero, sizeof(int), hipMemcpyHostToDevice));
    }
    s->chunk_h = s->chunk_f = 0;   // alone again: its own automatic item heights
    s->group = nullptr;
    s->group_slot = -1;
    drop_step_graphs(s);
    g->sims[slot] = nullptr;
    g->dirty = true;
    bool any = false;
    for (lb_sim* m : g->sims) any = any || m;
    if (!any) { g->storage = -1; g->thermal = -1; }
    return poll_flag(s);   // what the group's launches left in its flag
}

int lb_group_set_chunk(lb_group* g, int32_t rows) {
    if (!g) return fail(LB_EINVAL, "lb_group_set_chunk: NULL group");
    if (rows < 0) return fail(LB_EINVAL, "lb_group_set_chunk: rows must be >= 0 (0: automatic)");
    g->chunk = rows;
    g->dirty = true;
    return LB_OK;
}

int lb_group_step(lb_group* g, int64_t nsteps) {
    if (!g) return fail(LB_EINVAL, "lb_group_step: NULL group");
    if (nsteps < 0) return fail(LB_EINVAL, "lb_group_step: negative step count");
    if (nsteps == 0) return LB_OK;
    if (g->dirty) {
        if (int rc = group_rebuild(g)) return rc;
    }
    if (g->n_items == 0) return LB_OK;
    if (!g->exec || g->exec_steps != nsteps) {
        group_drop_graph(g);
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
        hipError_t e = group_enqueue(g, nsteps);
        hipError_t e2 = hipStreamEndCapture(g->stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(LB_EDEVICE, "lb_group_step: graph capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g->exec = nullptr;
            return fail(LB_EDEVICE, "lb_group_step: graph instantiation failed: %s", hipGetErrorString(e));
        }
        g->exec_steps = nsteps;
    }
    HIP_TRY(hipGraphLaunch(g->exec, g->stream));
    return LB_OK;
}

int lb_group_sync(lb_group* g) {
    if (!g) return fail(LB_EINVAL, "lb_group_sync: NULL group");
    HIP_TRY(hipStreamSynchronize(g->stream));
    return LB_OK;
}

int lb_group_remaining(lb_group* g, int64_t* left) {
    if (!g || !left) return fail(LB_EINVAL, "lb_group_remaining: NULL argument");
    HIP_TRY(hipMemcpyAsync(left, g->d_left, sizeof(int64_t) * g->max_sims, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return LB_OK;
}

}  // extern "C"

// ===================================================================== 3D ==

struct lb3_sim {
    lb3_params p{};
    int nsp = 1;
    int64_t cells = 0;
    size_t elem = 8, state_bytes = 0;
    hipStream_t stream = nullptr;
    void* A = nullptr;        // current state
    void* B = nullptr;        // predictor / next state
    void* phi[2] = {nullptr, nullptr};  // brackets of the moving populations, [nsp * 18][cells]
    int phi_cur = 0;          // phi[phi_cur] feeds the next pass
    bool phi_ok = false;      // it holds the brackets of the current state (left by the tiled update)
    void* metric = nullptr;   // flux stencils: pass 0 (x, y, z), pass 1 (x, y, z), [n][8] each
    double* dxyz = nullptr;   // cell widths dx[nx], dy[ny], dz[nz]
    double* partial = nullptr;
    double* dout = nullptr;
    std::vector<double> faces[3];
    size_t coef_off[2][3] = {{0, 0, 0}, {0, 0, 0}};
    bool has_grid = false, has_init = false, unstable = false;
    bool timing = false;
    int gather = 0;           // update kernel: 0 LDS tiles, 1 one thread per cell
    std::vector<hipEvent_t> events;
    std::vector<int> kinds;
    size_t n_rec = 0;
    int64_t launches[2] = {0, 0};
    double ms[2] = {0, 0};
};

namespace {

void release3(lb3_sim* s) {
    for (void* q : {s->A, s->B, s->phi[0], s->phi[1], s->metric, static_cast<void*>(s->dxyz), static_cast<void*>(s->partial),
                    static_cast<void*>(s->dout)})
        if (q) (void)hipFree(q);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    s->events.clear();
}

// the 2D stage-constant builder from the 3D parameters
lb_params as2d(const lb3_params& q) {
    lb_params p{};
    p.scheme = q.scheme;
    p.storage = q.storage;
    p.thermal = q.thermal;
    p.dt = q.dt;
    p.tau = q.tau;
    p.tau_g = q.tau_g;
    p.ax = q.a[0];
    p.ay = q.a[1];
    p.beta_g = q.beta_g;
    p.T0 = q.T0;
    p.rho_ref = q.rho_ref;
    p.T_ref = q.T_ref;
    return p;
}

Aux3Args aux3_args(const lb3_sim* s) {
    Aux3Args a{};
    a.state = s->A;
    a.n[0] = s->p.nx;
    a.n[1] = s->p.ny;
    a.n[2] = s->p.nz;
    a.cells = s->cells;
    a.thermal = s->p.thermal;
    a.hdt = s->p.scheme == LB_FV_EULER ? 0.0 : 0.5 * s->p.dt;
    for (int d = 0; d < 3; ++d) a.a[d] = s->p.a[d];
    a.bg = s->p.thermal ? s->p.beta_g : 0.0;
    a.T0 = s->p.T0;
    a.ref_f = s->p.storage == LB_F64 ? 0.0 : s->p.rho_ref;
    a.ref_g = s->p.storage == LB_F64 ? 0.0 : s->p.T_ref;
    a.dx = s->dxyz;
    a.dy = s->dxyz + s->p.nx;
    a.dz = s->dxyz + s->p.nx + s->p.ny;
    return a;
}

template <class R>
Fv3Args<R> fv3_args(const lb3_sim* s, const void* src, void* dst, const void* aux, bool corrector) {
    Fv3Args<R> a{};
    a.src = src;
    a.dst = dst;
    a.aux = aux;
    a.phi = static_cast<R*>(s->phi[s->phi_cur]);
    a.phi_next = s->gather ? nullptr : static_cast<R*>(s->phi[s->phi_cur ^ 1]);
    a.stage = s->gather || !s->phi_ok;
    a.n[0] = s->p.nx;
    a.n[1] = s->p.ny;
    a.n[2] = s->p.nz;
    for (int d = 0; d < 3; ++d) {
        a.wall[d] = s->p.bc[d] == LB_WALL;
        a.coef[d] = static_cast<const R*>(s->metric) + s->coef_off[corrector ? 1 : 0][d];
    }
    a.cells = s->cells;
    fill_stage_k<R>(as2d(s->p), a.k);
    a.az = R(s->p.a[2]);
    a.Tb = R(s->p.T_bottom);
    a.Tt = R(s->p.T_top);
    a.gather = s->gather;
    return a;
}

int record3(lb3_sim* s, int kind) {
    if (!s->timing) return LB_OK;
    if (s->n_rec == s->events.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        s->events.push_back(e);
        s->kinds.push_back(-1);
    }
    HIP_TRY(hipEventRecord(s->events[s->n_rec], s->stream));
    s->kinds[s->n_rec] = kind;
    ++s->n_rec;
    return LB_OK;
}

int fold3(lb3_sim* s) {
    if (s->n_rec == 0) return LB_OK;
    HIP_TRY(hipEventSynchronize(s->events[s->n_rec - 1]));
    for (size_t k = 0; k + 1 < s->n_rec; ++k) {
        const int kind = s->kinds[k];
        if (kind < 0 || kind > 1) continue;
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, s->events[k], s->events[k + 1]));
        s->ms[kind] += t;
        s->launches[kind] += 1;
    }
    s->n_rec = 0;
    return LB_OK;
}

int fv3_pass(lb3_sim* s, const void* src, void* dst, const void* aux, bool corrector) {
    if (int rc = record3(s, corrector ? 1 : 0)) return rc;
    hipError_t e;
    if (s->p.storage == LB_F64) {
        Fv3Args<double> a = fv3_args<double>(s, src, dst, aux, corrector);
        e = launch_fv3(s->p.storage, s->p.thermal, corrector, &a, s->stream);
    } else {
        Fv3Args<float> a = fv3_args<float>(s, src, dst, aux, corrector);
        e = launch_fv3(s->p.storage, s->p.thermal, corrector, &a, s->stream);
    }
    if (e != hipSuccess) {
        s->phi_ok = false;
        return fail(LB_EDEVICE, "3D FV launch failed: %s", hipGetErrorString(e));
    }
    if (!s->gather) s->phi_cur ^= 1;   // the tiled update left the brackets of dst there
    s->phi_ok = !s->gather;
    return LB_OK;
}

int check3(const lb3_sim* s) { return s ? LB_OK : fail(LB_EINVAL, "NULL handle"); }

}  // namespace

extern "C" {

int lb3_create(const lb3_params* p, lb3_sim** out) {
    try {
        if (!p || !out) return fail(LB_EINVAL, "lb3_create: NULL argument");
        *out = nullptr;
        if (p->nx < 4 || p->ny < 4 || p->nz < 4) return fail(LB_EINVAL, "lb3_create: nx, ny and nz must be >= 4");
        if (p->scheme != LB_FV_HEUN && p->scheme != LB_FV_SEMI && p->scheme != LB_FV_EULER)
            return fail(LB_EINVAL, "lb3_create: the 3D step has the FV schemes only");
        if (p->storage != LB_F64 && p->storage != LB_F32) return fail(LB_EINVAL, "lb3_create: storage must be LB_F64 or LB_F32");
        if (!(p->tau > 0) || (p->thermal && !(p->tau_g > 0)) || !(p->dt > 0))
            return fail(LB_EINVAL, "lb3_create: tau, tau_g and dt must be > 0");
        for (int d = 0; d < 3; ++d)
            if (p->bc[d] != LB_PERIODIC && p->bc[d] != LB_WALL) return fail(LB_EINVAL, "lb3_create: bad boundary kind");
        lb3_sim* s = new (std::nothrow) lb3_sim();
        if (!s) return fail(LB_ENOMEM, "lb3_create: out of host memory");
        s->p = *p;
        s->nsp = p->thermal ? 2 : 1;
        s->cells = int64_t(p->nx) * p->ny * p->nz;
        s->elem = p->storage == LB_F64 ? 8 : 4;
        s->state_bytes = size_t(s->nsp) * 19 * size_t(s->cells) * s->elem;
        s->stream = static_cast<hipStream_t>(p->stream);
        hipError_t e;
        if ((e = hipMalloc(&s->A, s->state_bytes)) != hipSuccess || (e = hipMalloc(&s->B, s->state_bytes)) != hipSuccess ||
            (e = hipMalloc(&s->phi[0], size_t(s->nsp) * 18 * size_t(s->cells) * s->elem)) != hipSuccess ||
            (e = hipMalloc(&s->phi[1], size_t(s->nsp) * 18 * size_t(s->cells) * s->elem)) != hipSuccess ||
            (e = hipMalloc(&s->partial, sizeof(double) * DIAG_BLOCKS * D_COUNT)) != hipSuccess ||
            (e = hipMalloc(&s->dout, sizeof(double) * D_COUNT)) != hipSuccess) {
            release3(s);
            delete s;
            return fail(e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE, "lb3_create: device allocation failed: %s",
                        hipGetErrorString(e));
        }
        *out = s;
        return LB_OK;
    } catch (...) {
        return fail(LB_ENOMEM, "lb3_create: unexpected failure");
    }
}

void lb3_destroy(lb3_sim* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    release3(s);
    delete s;
}

int lb3_set_grid(lb3_sim* s, const double* xf, int64_t nxf, const double* yf, int64_t nyf, const double* zf,
                 int64_t nzf) {
    if (int rc = check3(s)) return rc;
    try {
        const double* f[3] = {xf, yf, zf};
        const int64_t nf[3] = {nxf, nyf, nzf};
        const int n[3] = {s->p.nx, s->p.ny, s->p.nz};
        for (int d = 0; d < 3; ++d) {
            if (!f[d] || nf[d] != n[d] + 1) return fail(LB_EINVAL, "lb3_set_grid: need n+1 faces per axis");
            for (int64_t i = 0; i + 1 < nf[d]; ++i)
                if (!(f[d][i + 1] > f[d][i])) return fail(LB_EINVAL, "lb3_set_grid: faces not increasing");
        }
        std::vector<double> m, dxyz;
        for (int pass = 0; pass < 2; ++pass) {
            const double factor = pass == 0 ? s->p.dt : 0.5 * s->p.dt;
            for (int d = 0; d < 3; ++d) {
                std::vector<double> faces(f[d], f[d] + nf[d]);
                std::vector<double> w = quick_weights(faces, s->p.bc[d] == LB_PERIODIC);
                std::vector<double> st = flux_stencils(faces, w, factor);
                s->coef_off[pass][d] = m.size();
                m.insert(m.end(), st.begin(), st.end());
            }
        }
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < n[d]; ++i) dxyz.push_back(f[d][i + 1] - f[d][i]);
        std::vector<float> mf;
        if (s->p.storage != LB_F64) mf.assign(m.begin(), m.end());
        const void* mh = s->p.storage == LB_F64 ? static_cast<const void*>(m.data()) : mf.data();
        const size_t mbytes = s->p.storage == LB_F64 ? m.size() * sizeof(double) : mf.size() * sizeof(float);
        // the new grid goes to new buffers; the old one stays in use if this fails
        void* metric = nullptr;
        void* dxyz_d = nullptr;
        if (int rc = upload_all({{&metric, mh, mbytes}, {&dxyz_d, dxyz.data(), dxyz.size() * sizeof(double)}},
                                "lb3_set_grid"))
            return rc;
        if (hipError_t e = hipStreamSynchronize(s->stream); e != hipSuccess) {
            (void)hipFree(metric);
            (void)hipFree(dxyz_d);
            return fail(LB_EDEVICE, "set_grid: %s", hipGetErrorString(e));
        }
        if (s->metric) (void)hipFree(s->metric);
        if (s->dxyz) (void)hipFree(s->dxyz);
        s->metric = metric;
        s->dxyz = static_cast<double*>(dxyz_d);
        for (int d = 0; d < 3; ++d) s->faces[d].assign(f[d], f[d] + nf[d]);
        s->has_grid = true;
        return LB_OK;
    } catch (...) {
        return fail(LB_ENOMEM, "lb3_set_grid: out of host memory");
    }
}

int lb3_init(lb3_sim* s, const double* rho, const double* ux, const double* uy, const double* uz, const double* T) {
    if (int rc = check3(s)) return rc;
    if (!s->has_grid) return fail(LB_ESTATE, "lb3_init: call lb3_set_grid first");
    if (!rho || !ux || !uy || !uz || (s->p.thermal && !T)) return fail(LB_EINVAL, "lb3_init: NULL field");
    const size_t n = size_t(s->cells);
    double* d[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    const double* h[5] = {rho, ux, uy, uz, s->p.thermal ? T : rho};
    int rc = LB_OK;
    for (int q = 0; q < 5 && rc == LB_OK; ++q) rc = upload_temp(h[q], n, &d[q], s->stream);
    if (rc == LB_OK) {
        const double* in[5] = {d[0], d[1], d[2], d[3], d[4]};
        hipError_t e = launch_aux3(s->p.storage, 0, aux3_args(s), in, nullptr, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) rc = fail(LB_EDEVICE, "lb3_init: %s", hipGetErrorString(e));
    }
    for (double* q : d) if (q) (void)hipFree(q);
    s->phi_ok = false;   // brackets of the old state, if any
    if (rc == LB_OK) { s->has_init = true; s->unstable = false; }
    return rc;
}

int lb3_step(lb3_sim* s, int64_t nsteps) {
    if (int rc = check3(s)) return rc;
    if (!s->has_init) return fail(LB_ESTATE, "lb3_step: call lb3_init first");
    if (nsteps < 0) return fail(LB_EINVAL, "lb3_step: negative step count");
    if (s->unstable) return fail(LB_EUNSTABLE, "lb3_step: non-finite populations were detected");
    for (int64_t n = 0; n < nsteps; ++n) {
        int rc;
        if (s->p.scheme == LB_FV_HEUN) {
            if ((rc = fv3_pass(s, s->A, s->B, nullptr, false))) return rc;  // f~* -> B
            if ((rc = fv3_pass(s, s->B, s->A, s->A, true))) return rc;      // corrector in place over A
        } else {
            if ((rc = fv3_pass(s, s->A, s->B, nullptr, false))) return rc;
            std::swap(s->A, s->B);
        }
    }
    if (s->timing) return record3(s, -1);
    return LB_OK;
}

int lb3_sync(lb3_sim* s) {
    if (int rc = check3(s)) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return LB_OK;
}

int lb3_moments(lb3_sim* s, double* rho, double* ux, double* uy, double* uz, double* T) {
    if (int rc = check3(s)) return rc;
    if (!s->has_init) return fail(LB_ESTATE, "lb3_moments: no state");
    const size_t n = size_t(s->cells);
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, 5 * n * sizeof(double)));
    double* outs[5] = {d, d + n, d + 2 * n, d + 3 * n, d + 4 * n};
    hipError_t e = launch_aux3(s->p.storage, 1, aux3_args(s), nullptr, outs, s->stream);
    double* h[5] = {rho, ux, uy, uz, T};
    for (int q = 0; q < 5 && e == hipSuccess; ++q)
        if (h[q]) e = hipMemcpyAsync(h[q], outs[q], n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb3_moments: %s", hipGetErrorString(e));
    return LB_OK;
}

int lb3_get_populations(lb3_sim* s, double* f, double* g) {
    if (int rc = check3(s)) return rc;
    if (!s->has_init) return fail(LB_ESTATE, "lb3_get_populations: no state");
    if (!f) return fail(LB_EINVAL, "lb3_get_populations: NULL f");
    const size_t n = size_t(s->cells) * 19;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, size_t(s->nsp) * n * sizeof(double)));
    double* outs[1] = {d};
    hipError_t e = launch_aux3(s->p.storage, 2, aux3_args(s), nullptr, outs, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && s->p.thermal && g) e = hipMemcpyAsync(g, d + n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb3_get_populations: %s", hipGetErrorString(e));
    return LB_OK;
}

int lb3_diagnostics(lb3_sim* s, double* out) {
    if (int rc = check3(s)) return rc;
    if (!s->has_init) return fail(LB_ESTATE, "lb3_diagnostics: no state");
    if (!out) return fail(LB_EINVAL, "lb3_diagnostics: NULL output");
    Diag3Args d{};
    d.a = aux3_args(s);
    const int nz = s->p.nz;
    const auto& zf = s->faces[2];
    const double H = zf[nz] - zf[0], dT = s->p.T_bottom - s->p.T_top;
    d.walls = s->p.thermal && s->p.bc[2] == LB_WALL && dT != 0.0;
    if (d.walls) {
        d_weights(zf[0], 0.5 * (zf[0] + zf[1]), 0.5 * (zf[1] + zf[2]), d.nub);
        d_weights(zf[nz], 0.5 * (zf[nz - 1] + zf[nz]), 0.5 * (zf[nz - 2] + zf[nz - 1]), d.nut);
        d.nu_scale = -H / dT;
    }
    d.Tb = s->p.T_bottom;
    d.Tt = s->p.T_top;
    d.inv_area = 1.0 / ((s->faces[0].back() - s->faces[0][0]) * (s->faces[1].back() - s->faces[1][0]));
    hipError_t e = launch_diag3(s->p.storage, d, s->partial, s->dout, s->stream);
    double o[D_COUNT];
    if (e == hipSuccess) e = hipMemcpyAsync(o, s->dout, sizeof o, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb3_diagnostics: %s", hipGetErrorString(e));
    const double kappa = s->p.tau_g / 3.0;
    out[0] = o[D_MASS];
    out[1] = o[D_EKIN];
    out[2] = o[D_ETH];
    out[3] = d.walls ? o[D_NUB] : 0.0;
    out[4] = d.walls ? o[D_NUT] : 0.0;
    out[5] = d.walls ? 1.0 + H * (o[D_UT] / o[D_VOL]) / (kappa * dT) : 0.0;
    out[6] = o[D_VOL];
    out[7] = o[D_BAD];
    if (o[D_BAD] != 0.0) s->unstable = true;
    return LB_OK;
}

int lb3_set_update(lb3_sim* s, int kind) {
    if (int rc = check3(s)) return rc;
    if (kind != 0 && kind != 1) return fail(LB_EINVAL, "lb3_set_update: kind must be 0 (tiles) or 1 (per cell)");
    s->gather = kind;
    s->phi_ok = false;
    return LB_OK;
}

int lb3_set_timing(lb3_sim* s, int on) {
    if (int rc = check3(s)) return rc;
    if (s->timing && !on)
        if (int rc = fold3(s)) return rc;
    s->timing = on != 0;
    s->launches[0] = s->launches[1] = 0;
    s->ms[0] = s->ms[1] = 0;
    s->n_rec = 0;
    return LB_OK;
}

int lb3_kernel_times(lb3_sim* s, int64_t* launches, double* ms) {
    if (int rc = check3(s)) return rc;
    if (!launches || !ms) return fail(LB_EINVAL, "lb3_kernel_times: NULL output");
    if (int rc = fold3(s)) return rc;
    for (int k = 0; k < 2; ++k) { launches[k] = s->launches[k]; ms[k] = s->ms[k]; }
    return LB_OK;
}

}  // extern "C"
