// Kernel argument blocks and launchers of liblb (host and device visible).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_device.h"

namespace lbk {

enum Storage { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2, ST_F16 = 3 };

// Width in lanes of the FV strip kernel: 252 owned columns + 2 halo columns
// on each side.  One lane per column, the block marches up its rows.
constexpr int FV_LANES = 256;
constexpr int FV_HALO = 2;

// Per-face QUICK weights (sec. 2.2.3), face k between cells k-1 and k:
//   c.n > 0 : P = k-1, E = k, W = k-2   ->  up[0] P + up[1] E + up[2] W
//   c.n < 0 :                EE = k+1   ->  dn[0] E + dn[1] P + dn[2] EE
// stored as 6 numbers per face: up0 up1 up2 dn0 dn1 dn2, with
//   up = (1 - g1 + g2, g1, -g2), dn = (1 - g3 + g4, g3, -g4).
template <class R>
struct Metric {
    const R* xw;   // [(nx+1)*6]
    const R* yw;   // [(ny+1)*6]
    const R* idx;  // [nx]  1/dx (S/V of the x faces)
    const R* idy;  // [ny]
};

template <class R>
struct FvArgs {
    const void* src;  // state read with halo: f~n (predictor, single pass) or f~* (corrector)
    const void* loc;  // corrector only: f~n, read at the cell itself
    void* dst;        // output state
    int nx, ny;
    int64_t plane;    // nx * ny
    int wall_x, wall_y;
    int strip_w;      // owned columns per strip (<= FV_LANES - 4)
    int chunk_h;      // rows per chunk
    Metric<R> m;
    StageConst<R> k;
    R dt_update;      // dt (predictor / single pass) or dt/2 (corrector)
    R T_bottom, T_top;
    R ref_f, ref_g;   // storage offsets (rho_ref, T_ref)
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
};

// Host launchers (defined in the .hip files).  `storage` selects the
// template instance; every launcher returns the hipError_t of the launch.
hipError_t launch_fv_pass(int storage, bool thermal, bool corrector, const void* args,
                          int n_strips, int n_chunks, hipStream_t s);
hipError_t launch_st(int storage, bool thermal, bool stream_only, const StArgs& a, hipStream_t s);

struct AuxArgs {
    void* state;       // populations (f planes then g planes)
    int nx, ny;
    int64_t plane;
    int thermal;
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
hipError_t launch_diagnostics(int storage, const DiagArgs& d, double* partial, double* out,
                              hipStream_t s);

}  // namespace lbk
