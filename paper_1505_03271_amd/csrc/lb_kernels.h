// Kernel argument blocks and launchers of liblb (host and device visible).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_device.h"

namespace lbk {

enum Storage { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2, ST_F16 = 3, ST_BF16S = 4, ST_F16S = 5 };

// Lanes of an FV block (one lane per column, a work item marches up its
// rows): a wide item owns FV_LANES - 4 columns + 2 halo columns on each side;
// in narrow mode a block runs four items of FV_NARROW lanes, one per wave.
constexpr int FV_LANES = 256;
constexpr int FV_NARROW = 64;
constexpr int FV_HALO = 2;
// The fused step (predictor and corrector in one launch) forms f~* two cells
// beyond its strip, so it reads f~n with a halo of four.
constexpr int FV_FUSED_HALO = 4;

// Stage constants of the FV kernel in offset arithmetic (see fv.hip), with
// d = p - w ref, poly = f_eq/(w rho), frc = F/(w rho):
//   bracket   phi - w ref = omk1 d + w (k1 (rho - ref) + rho (k1 (poly - 1) + kh frc))   (f)
//             phi - w Tr  = omk1g d + k1g w ((T - Tr) + T (poly - 1))                       (g)
//   f~ + C    b           = omkc d + w (kc (rho - ref) + rho (kc (poly - 1) + kf frc))
//             b           = omkcg d + kcg w ((T - Tr) + T (poly - 1))
// k1x3 = 3 k1 etc.
template <class R>
struct StageK {
    R hdt, ax, ay, bg, T0, ref_f, ref_g;
    R k1, kh, k1x3, khx3, omk1, k1g, omk1g;
    R kc, kf, kcx3, kfx3, omkc, omkcg, kcg;
    R cP, cB;   // force weights of the split stage: kh - (1 - k1) hdt, kf - (1 - kc) hdt
};

template <class R>
struct FvArgs {
    const void* src;   // state read with halo: f~n (predictor / single pass / fused step) or f~* (corrector)
    void* dst;         // output state (fused step: f~n+1)
    void* aux;         // corrector: the input f~n (read only); NULL otherwise
    const R* xcoef2;   // fused step: the corrector's weights (xcoef, ycoef: the predictor's)
    const R* ycoef2;
    uint32_t state_bytes;  // whole state (grouped layout, see pop_index; or SplitLayout)
    uint32_t group_bytes;  // one group plane: 4 elements per cell (split: 8 bytes per cell)
    uint32_t rest_off;     // byte offset of the rest plane (unused by split states)
    int nx, ny;
    int wall_x, wall_y;  // 0 periodic, 1 no-slip wall, 2 (x only) fixed density
    int strip_w;       // owned columns per strip (FV_LANES - 4, or FV_NARROW - 4 in narrow mode)
    int narrow;        // 1: four FV_NARROW-lane items per block
    int chunk_h;       // rows per chunk
    int n_strips, n_items;  // work items: n_strips * n_chunks, chunk-major
    const R* xcoef;    // [nx][8] four-point flux weights (c>0: i-2..i+1, c<0: i-1..i+2), times dt or dt/2
    const R* ycoef;    // [ny][8]
    StageK<R> k;
    R Tb, Tt;          // wall temperatures (bottom, top) for the isothermal anti-reflection of g
    R rho_x0, rho_x1;  // densities on the x faces of a fixed-density axis
    const R* tref;     // per-row thermal reference (g stored as g - w_a tref[row]), or NULL: k.ref_g
    const R* qref;     // split thermal storage: per-row heat-flux reference, the stored g residual is
                       // r_a - w_a c_ay qref[row] (NULL: 0)
    int* bad;          // set to 1 when a stored cell is not finite (NULL: no check); the serving
                       // kernel skips a simulation whose flag is set
};

struct StArgs {
    const void* src;
    void* dst;
    int nx, ny;
    int64_t plane;
    int wall_x, wall_y;
    double tau, tau_g;   // paper's tau; tau~ = tau + 1/2
    double ax, ay, bg, T0, T_bottom, T_top;
    double ref_f, ref_g;
    const float* tref;   // per-row thermal reference of the stored g, or NULL
    int pairs;           // FP32 or 16-bit storage, even nx: two cells per thread (st_step_pair)
    int* bad;            // set to 1 when a collided cell is not finite (NULL: no check)
};

// Host launchers (defined in the .hip files).  `storage` selects the
// template instance; every launcher returns the hipError_t of the launch.
hipError_t launch_fv_pass(int storage, bool thermal, bool corrector, const void* args, hipStream_t s);
// One fused step (x periodic): args as for the predictor (src f~n, dst f~n+1),
// plus the corrector's weights in xcoef2 / ycoef2.
hipError_t launch_fv_fused(int storage, bool thermal, const void* args, hipStream_t s);
int fv_fused_resident_blocks(int storage, bool thermal);
// Serving: one launch over the work items of many simulations.  args holds
// 2 FvArgs per simulation (predictor, corrector); items are (simulation,
// local item), the n_wide items of wide-strip members first, then the
// n_narrow items of narrow-strip members; left[s] is the number of steps
// simulation s still has to do.
hipError_t launch_fv_multi(int storage, bool thermal, bool corrector, const void* args, const int2* items,
                           int n_wide, int n_narrow, const int64_t* left, hipStream_t s);
// Serving, fused steps: args holds 2 FvArgs per simulation (its state in the
// first / second buffer of its pair), phase[s] which of the two applies.
hipError_t launch_fv_fused_multi(int storage, bool thermal, const void* args, const int2* items, int n_items,
                                 const int64_t* left, const int* phase, hipStream_t s);
// left[i] -= 1 where positive, and then phase[i] ^= 1 (phase != NULL); with
// every != NULL also the renewal count since[i] of the thermal references
// and due[i] (1: renew after this step).
hipError_t launch_tick(int64_t* left, int n, const int64_t* every, int64_t* since, int* due, int* phase,
                       hipStream_t s);
size_t fv_args_bytes(int storage);

// Largest number of FV blocks of one launch that are resident at once.
int fv_resident_blocks(int storage, bool thermal, bool corrector);
hipError_t launch_st(int storage, bool thermal, bool stream_only, const StArgs& a, hipStream_t s);

struct AuxArgs {
    void* state;       // populations (layout: pop_index)
    int nx, ny;
    int64_t plane;
    int thermal;
    int grouped;       // 1: grouped layout (FV schemes), 0: SoA (ST)
    const float* tref; // per-row thermal reference of the stored g, or NULL: ref_g
    const float* qref; // split thermal storage: per-row heat-flux reference of the g residuals, or NULL
    double hdt;        // velocity shift dt/2 (0 for Euler)
    double ax, ay, bg, T0;
    double ref_f, ref_g;
    const double* dx;  // [nx] cell widths
    const double* dy;  // [ny]
};

hipError_t launch_init(int storage, const AuxArgs& a, const double* rho, const double* ux,
                       const double* uy, const double* T, hipStream_t s);
hipError_t launch_moments(int storage, const AuxArgs& a, double* rho, double* ux, double* uy,
                          double* T, hipStream_t s);
hipError_t launch_get_pops(int storage, const AuxArgs& a, double* out, hipStream_t s);
hipError_t launch_set_pops(int storage, const AuxArgs& a, const double* in, hipStream_t s);
// New per-row thermal references = row means of T (and, for split storage,
// heat-flux references = row means of the g residuals' vertical flux); the
// stored g re-encoded.
hipError_t launch_rebase(int storage, const AuxArgs& a, hipStream_t s);
// The same for the rows items[q] = (simulation, row) of the simulations
// whose due flag is set (args: two AuxArgs per simulation, its state in the
// first or the second buffer of its pair, chosen by phase[simulation], or
// the first when phase is NULL; device memory).
hipError_t launch_rebase_multi(int storage, const AuxArgs* args, const int2* items, int n_items, const int* due,
                               const int* phase, hipStream_t s);

// Diagnostics: per-block FP64 partial sums, then one block folds them in a
// fixed order (bit-reproducible).  Output slots:
enum { D_MASS, D_EKIN, D_ETH, D_NUB, D_NUT, D_UT, D_VOL, D_BAD, D_COUNT };
struct DiagArgs {
    AuxArgs a;
    double nub[3], nut[3];  // one-sided derivative weights (wall value, first, second cell)
    double Tb, Tt;
    double inv_Lx;           // 1 / (x extent) for the wall averages
    double nu_scale;         // -H / dT
    int walls;               // thermal with y walls: compute the wall Nusselt sums
};
constexpr int DIAG_BLOCKS = 1024;
// Per-row x averages (one block per row, fixed reduction order):
// out[q * ny + j], q = 0 <T>, 1 <T^2>, 2 <ux^2>, 3 <uy^2>, 4 <uy T>, weighted by dx / Lx.
constexpr int PROFILE_ROWS = 5;
hipError_t launch_profiles(int storage, const AuxArgs& a, double inv_Lx, double* out, hipStream_t s);
// Post-processing of the folded sums into lb_diagnostics' values, on the
// device (finish = 1): the wall Nusselt slots are zeroed without isothermal
// walls, and slot D_UT becomes Nu_vol = 1 + H (sum V u_y T / sum V) / (kappa dT).
struct DiagFinal {
    int finish, walls;
    double H, kappa, dT;
};
// Partial sums used for a grid of `cells` cells: diag_blocks(cells) * D_COUNT doubles.
int diag_blocks(int64_t cells);
hipError_t launch_diagnostics(int storage, const DiagArgs& d, double* partial, double* out,
                              hipStream_t s, const DiagFinal& fin);

// ---- three dimensions (D3Q19, fv3d.hip) ----------------------------------
template <class R>
struct Fv3Args {
    const void* src;   // state read by the stage and at the own cell (f~n, or f~* in the corrector)
    void* dst;         // new state
    const void* aux;   // corrector: f~n at the own cell; NULL otherwise
    R* phi;            // scratch: [nsp * 18][cells] brackets of src
    R* phi_next;       // tiled update: where to put the brackets of dst for the next pass, or NULL
    int stage;         // 1: compute phi from src first (stage kernel); 0: phi already holds them
    int n[3];
    int wall[3];       // per axis: 0 periodic, 1 wall
    int64_t cells;
    const R* coef[3];  // per axis [n][8] four-point stencils (c > 0: i-2..i+1, c < 0: i-1..i+2), times dt or dt/2
    StageK<R> k;       // stage constants (k.ax, k.ay: x and y accelerations)
    R az;              // constant z acceleration (the Boussinesq term is added along z)
    R Tb, Tt;          // z wall temperatures
    int gather;        // update kernel: 0 tiles staged in LDS, 1 one thread per cell with direct loads
    int* bad;          // set to 1 when a cell's density or temperature is not finite (NULL: no check)
};
// One FV stage (stage + update kernels) of a 3D simulation.
hipError_t launch_fv3(int storage, bool thermal, bool corrector, const void* args, hipStream_t s);
size_t fv3_args_bytes(int storage);

struct Aux3Args {
    void* state;       // (s * 19 + a) * cells + cell
    int n[3];
    int64_t cells;
    int thermal;
    double hdt, a[3], bg, T0, ref_f, ref_g;
    const double *dx, *dy, *dz;
};
// what: 0 init (in = rho, ux, uy, uz, T), 1 moments (out = rho, ux, uy, uz, T),
// 2 populations (out[0] = [nsp * 19][cells] in double)
hipError_t launch_aux3(int storage, int what, const Aux3Args& a, const double* const* in, double* const* out,
                       hipStream_t s);
struct Diag3Args {
    Aux3Args a;
    double nub[3], nut[3];   // one-sided derivative weights at the z walls
    double Tb, Tt, inv_area, nu_scale;
    int walls;
};
hipError_t launch_diag3(int storage, const Diag3Args& d, double* partial, double* out, hipStream_t s);

// Streaming-bandwidth reference sweeps (probe.hip): kind 0 copy, 1 two reads
// and a write, 2 two reads; n elements of 16 bytes per buffer, 256 lanes per
// block.
hipError_t launch_stream(int kind, int grid, const void* a, const void* b, void* d, size_t n, hipStream_t s);

}  // namespace lbk
