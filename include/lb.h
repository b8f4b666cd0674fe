/*
 * liblb: finite-volume and streaming lattice Boltzmann time steps on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Shrestha, Mompean & Calzavarini, "Finite Volume vs. Streaming-based
 * Lattice Boltzmann algorithm for fluid-dynamics simulations: a one-to-one
 * accuracy and performance study" (arXiv:1505.03271).
 *
 *   FV step   sec. 2.2: cell-centred finite volumes (eq:fv), semi-implicit
 *             collision (eq:semi) with a Heun predictor-corrector on the
 *             advection (eq:semi-heun), QUICK face values (sec. 2.2.3),
 *             Guo forcing (eq:F2), double-reflection no-slip walls
 *             ("Boundary conditions").
 *   ST step   sec. 2.1, eq:ST: collide and stream, dt = dx = 1, half-way
 *             bounce-back walls.
 *   Thermal   sec. 5, eq:LBg: second population set g with
 *             g_eq = (T/rho) f_eq, Boussinesq acceleration
 *             a = beta g (T - T0) along +y, isothermal walls at y = 0 (bottom)
 *             and y = H (top).
 *
 * Units are lattice units throughout.  tau is the paper's relaxation time
 * (nu = tau cs^2, cs^2 = 1/3); the library uses tau~ = tau + dt/2 internally.
 *
 * Populations: D2Q9, index a = 0..8 with velocities
 *   (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 * Field arrays crossing this interface are row-major [ny][nx] (x fastest);
 * population arrays are [9][ny][nx].
 *
 * Every function returns LB_OK (0) or an LB_E* code and never throws; the
 * message of the last error on the calling thread is lb_last_error().  A
 * handle must not be used from two threads at once; distinct handles are
 * independent.  Device work is enqueued on the handle's stream; functions
 * that return data to the host synchronise that stream first.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lb_status {
    LB_OK = 0,
    LB_EINVAL = 1,    /* bad argument: sizes, NULL pointers, tau <= 0, ... */
    LB_ENOMEM = 2,    /* device or host allocation failed */
    LB_EDEVICE = 3,   /* a HIP call failed (message has the HIP error) */
    LB_ESTATE = 4,    /* call out of order (e.g. lb_step before lb_init) */
    LB_EUNSTABLE = 5  /* a non-finite population was found (simulation blew up) */
};

enum lb_scheme {
    LB_FV_HEUN = 0,   /* eq:semi-heun: the paper's method */
    LB_FV_SEMI = 1,   /* eq:semi: semi-implicit collision, Euler advection */
    LB_FV_EULER = 2,  /* eq:euler: explicit Euler */
    LB_ST = 3         /* eq:ST: streaming, dt = dx = 1, uniform unit grid */
};

enum lb_storage {
    LB_F64 = 0,   /* double populations, double arithmetic (parity path) */
    LB_F32 = 1,   /* float offsets f - w rho_ref, float arithmetic */
    LB_BF16 = 2,  /* bfloat16 offsets (round to nearest even), float arithmetic */
    LB_F16 = 3,   /* IEEE half offsets (round to nearest even), float arithmetic */
    /* Moment-split storage, FV schemes only: per cell the conserved moments
     * (rho - rho_ref, j = sum c f~, T - T_row) in float and the residuals
     * f~ - (f_eq - dt/2 F) and g - g_eq of 6 + 8 populations in 16 bits (the
     * other residuals follow from zero mass and momentum), 44 bytes per
     * thermal cell.  Small per-step increments of the moments are kept at
     * float resolution where plain 16-bit offsets would round them away. */
    LB_BF16S = 4, /* residuals in bfloat16 */
    LB_F16S = 5   /* residuals in IEEE half, scaled by 2^10 */
};

enum lb_boundary {
    LB_PERIODIC = 0,
    LB_WALL = 1,   /* no-slip; for g isothermal on y walls, adiabatic on x walls */
    /* Fixed density ("Boundary conditions", second rule), x axis, FV schemes,
     * not thermal: the densities rho_x0 (face x_faces[0]) and rho_x1 (face
     * x_faces[nx]) are imposed by ghost populations equal to the mirror
     * cell's, rescaled by (2 rho_S - rho) / rho.  A density difference drives
     * a pressure-driven flow (p = cs^2 rho). */
    LB_DENSITY = 2
};

enum lb_flags {
    /* ST only: streaming without collision, moving raw stored words (the
     * thermal rule degenerates to plain bounce-back).  A check of the
     * streaming permutation, bit for bit. */
    LB_FLAG_STREAM_ONLY = 1
};

typedef struct lb_params {
    int32_t nx, ny;          /* cells along x and y, >= 4 */
    int32_t scheme;          /* enum lb_scheme */
    int32_t storage;         /* enum lb_storage */
    int32_t thermal;         /* 1: evolve g as well (sec. 5) */
    int32_t bc_x, bc_y;      /* enum lb_boundary */
    int32_t flags;           /* enum lb_flags */
    double dt;               /* time step (ignored by LB_ST, which uses 1) */
    double tau, tau_g;       /* paper's relaxation times, > 0 */
    double ax, ay;           /* constant body acceleration */
    double beta_g, T0;       /* Boussinesq: a_y += beta_g (T - T0) */
    double T_bottom, T_top;  /* wall temperatures at y = y_faces[0], y_faces[ny] */
    double rho_ref, T_ref;   /* storage offsets (LB_F32/BF16/F16): f - w rho_ref, g - w T_ref */
    double rho_x0, rho_x1;   /* LB_DENSITY on x: densities on the faces x_faces[0] and x_faces[nx] */
    void* stream;            /* hipStream_t to enqueue on, or NULL (null stream) */
} lb_params;

typedef struct lb_sim lb_sim;

/* Create a simulation.  The library owns the handle and all device buffers
 * (two population buffers of 9 or 18 planes each).  Errors: LB_EINVAL for
 * unsupported sizes/values (nx or ny < 4, tau or tau_g <= 0, dt <= 0 for FV,
 * one population buffer of 4 GiB or more (buffer offsets are 32 bits);
 * thermal with bc_y periodic is allowed but lb_nusselt then fails),
 * LB_ENOMEM, LB_EDEVICE. */
int lb_create(const lb_params* p, lb_sim** out);

/* Release the handle and its device memory (NULL is a no-op).  A group
 * member leaves its group first (as lb_group_remove). */
void lb_destroy(lb_sim* sim);

/* Grid (sec. 3, eq:grids; sec. 2.2.3).  x_faces[0..nx] and y_faces[0..ny]
 * are the cell-face coordinates, strictly increasing; cell centres are face
 * midpoints.  Copied; the caller keeps ownership.  The library derives 1/dx,
 * 1/dy and the QUICK coefficients gamma_1..4 of every face, with mirrored
 * ghost centres at walls and periodic images otherwise.  LB_ST requires unit
 * spacing (faces 0, 1, ..., n up to a common offset) or returns LB_EINVAL.
 * Must precede lb_init.  May be called again, between steps, for a new
 * grid; if that call fails the previous grid stays in use. */
int lb_set_grid(lb_sim* sim, const double* x_faces, int64_t n_xf,
                const double* y_faces, int64_t n_yf);

/* Face helpers (eq:grids), write n+1 faces on [0, L]. */
int lb_grid_uniform(int64_t n, double L, double* faces);
/* Hyperbolic tangent with the paper's factor s1 = tanh(stretch). */
int lb_grid_tanh(int64_t n, double L, double stretch, double* faces);
/* Hyperbolic sine with factor s2 (the paper uses 6.5); n must be even (the
 * two branches of eq:grids meet at i = n/2), else LB_EINVAL. */
int lb_grid_sinh(int64_t n, double L, double s2, double* faces);
/* Chebyshev faces xi_i = L/2 (1 - cos(i pi / n)), i = 0..n: the printed
 * form, with i - 1/2 in place of i, does not start at 0 nor end at L; this
 * reading keeps the nodes' spacing and spans [0, L]. */
int lb_grid_chebyshev(int64_t n, double L, double* faces);

/* Initial state at equilibrium (sec. 3.2, sec. 5): host arrays [ny][nx],
 * caller-owned; T is ignored (may be NULL) unless thermal.  Populations are
 * f~ = f_eq(rho, u) - dt/2 F(rho, u, a) and g~ = (T/rho) f_eq (appendix A),
 * so lb_moments returns the given fields.  LB_ESTATE without a grid. */
int lb_init(lb_sim* sim, const double* rho, const double* ux, const double* uy,
            const double* T);

/* Enqueue nsteps time steps (asynchronous).  Returns LB_EUNSTABLE if an
 * earlier check (lb_diagnostics or lb_nusselt) found non-finite
 * populations, LB_ESTATE before lb_init. */
int lb_step(lb_sim* sim, int64_t nsteps);

/* Wait for the handle's stream. */
int lb_sync(lb_sim* sim);

/* Macroscopic fields (eq:ST relations and "Force term"): rho = sum f~,
 * u = sum c f~ / rho + dt/2 a, T = sum g~.  Synchronises; writes caller-owned
 * host arrays [ny][nx] computed in double; any pointer may be NULL. */
int lb_moments(lb_sim* sim, double* rho, double* ux, double* uy, double* T);

/* Nusselt numbers (sec. 5): wall-averaged -H dT/dy / dT at the bottom and top
 * walls from the second-order one-sided difference through the wall value
 * and the first two cell centres, and the volume value
 * 1 + H <u_y T>_V / (kappa dT), kappa = tau_g / 3, dT = T_bottom - T_top.
 * FP64 reductions on the device.  LB_EINVAL unless thermal with y walls. */
int lb_nusselt(lb_sim* sim, double* nu_bottom, double* nu_top, double* nu_vol);

/* Horizontal (x) averages per row j, FP64 device reductions (sec. 5; the
 * paper time-averages them, which is left to the caller).  out is a
 * caller-owned host array [6][ny], n_out = 6 * ny:
 *   0  T_m(y)    = <T>_x
 *   1  T_rms(y)  = sqrt(<T^2>_x - <T>_x^2)
 *   2  <u_x^2>_x^(1/2),  3  <u_y^2>_x^(1/2)
 *   4  <u_y T>_x
 *   5  Nu(y) = (<u_y T>_x - kappa d<T>_x/dy) / (kappa dT / H), the
 *      derivative from the parabola through the neighbouring cell centres
 *      (through the wall value at the first and last row), kappa = tau_g/3.
 * x averages are weighted by the cell widths.  Rows 0, 1 and 4 are
 * filled for any thermal run; row 5 needs y walls at different
 * temperatures (else 0).  LB_EINVAL unless thermal or if n_out != 6 ny. */
int lb_profiles(lb_sim* sim, double* out, int64_t n_out);

/* FP64 device reductions, out[8]: mass sum V rho, kinetic sum V rho|u|^2/2,
 * thermal sum V T, Nu bottom, Nu top, Nu volume (0 if not applicable),
 * volume sum V, and 1.0 if any population is non-finite (which also makes
 * later lb_step calls return LB_EUNSTABLE). */
int lb_diagnostics(lb_sim* sim, double* out);

/* lb_diagnostics for callers that cannot allocate device memory or wait for
 * the device (code under HIP graph capture, tight serving loops): the same
 * eight values, written to out_device, a caller-owned DEVICE array of 8
 * doubles, by kernels enqueued on the handle's stream; the call returns at
 * once (no synchronisation, no device-to-host copy) and allocates nothing.
 * The partial sums go to a file-scope device array of DIAG_BLOCKS x 8
 * doubles (64 KiB) per GPU, held until the process ends; every grid fits it
 * (larger grids fold more cells per partial sum), and a call that would need
 * more is refused with LB_EINVAL.  All calls on one GPU share that array:
 * calls that overlap on one GPU (other streams, other threads) race, so
 * order them on one stream.  The handle's device must be current
 * (LB_EINVAL otherwise).  A member of a group that runs fused steps gets
 * LB_ESTATE (which of its buffers holds the state is known on the device
 * only; lb_diagnostics finds out).  Unlike lb_diagnostics it leaves the handle's
 * stability state alone: read the non-finite slot (out[7]) from the output. */
int lb_diagnostics_noalloc(lb_sim* sim, double* out_device);

/* Decoded populations in double, [9][ny][nx] for f and g (g may be NULL; it
 * is ignored unless thermal). */
int lb_get_populations(lb_sim* sim, double* f, double* g);
int lb_set_populations(lb_sim* sim, const double* f, const double* g);

/* Raw state (checkpoint), exactly lb_state_bytes() bytes: the stored words
 * of f then g, followed by the per-row references they are encoded with
 * (thermal non-F64 storage: T_ref[ny] floats; thermal split storage: then
 * the heat-flux reference q[ny] floats).  Restoring it and stepping is
 * bit-identical to not having stopped (the rebase countdown of
 * lb_set_rebase is not part of it). */
size_t lb_state_bytes(const lb_sim* sim);
int lb_get_state(lb_sim* sim, void* host, size_t bytes);
int lb_set_state(lb_sim* sim, const void* host, size_t bytes);

/* Kernel timing: when enabled, every launch made by lb_step is bracketed by
 * HIP events on the handle's stream (and lb_step launches every kernel
 * itself instead of replaying captured graphs).  lb_kernel_times
 * synchronises and returns, per kernel kind (0: FV predictor or single FV
 * pass, 1: FV corrector, 2: ST, 3: FV fused step), the number of launches
 * and their total milliseconds since the last reset (arrays of length 4). */
int lb_set_timing(lb_sim* sim, int enable);
int lb_kernel_times(lb_sim* sim, int64_t* launches, double* total_ms);

/* Thermal reference rows (non-F64 storage of a thermal run): the stored g
 * are offsets from w_a T_ref(row), T_ref(row) starting as the row means of
 * the initial temperature (lb_init).  Split storage (LB_BF16S, LB_F16S) has
 * a second row value, the heat-flux reference q(row), 0 at lb_init: the
 * stored g residual of population a is r_a - w_a c_ay q(row), so that the
 * 16 bits resolve departures from the row's mean vertical heat flux (the
 * conductive flux of a Rayleigh-Benard cell would otherwise set their
 * rounding step).  lb_rebase sets T_ref(row) to the current row means and
 * q(row) to 3 x the row mean of sum_a c_ay r_a, and re-encodes the stored g
 * (one rounding); with lb_set_rebase(every > 0) lb_step does this after
 * every `every` steps (0 never), and so do group steps for a member (its
 * count of steps since the last renewal goes with it into and out of the
 * group, so the result is the same alone and in a group).  The default is
 * 100 for split thermal storage, whose residuals would otherwise hold a
 * roll growing out of the conductive state below their rounding step, and
 * 0 otherwise.  No-ops for FP64 storage or isothermal runs. */
int lb_rebase(lb_sim* sim);
int lb_set_rebase(lb_sim* sim, int64_t every);

/* Lanes per work item of the FV kernels (a launch-shape knob): 256 (wide
 * strips of 252 columns, one item per block of 256 lanes), 64 (narrow
 * strips of 60 columns, four items per block, one per wave), or 0 (the
 * default: whichever needs fewer lanes for nx, narrow weighted 4% heavier).
 * Results are identical either way.  Resets a height set with
 * lb_set_fv_chunk.  LB_EINVAL for other values. */
int lb_set_fv_lanes(lb_sim* sim, int lanes);

/* ST with FP32 or 16-bit storage on grids of even nx (a launch-shape
 * knob): 1 (the default) two cells of a row per thread, each population of
 * both read as one 64- or 32-bit word and those that stay in their column
 * written as one; 0 one cell per thread.  Results are identical either
 * way.  LB_EINVAL for other values. */
int lb_set_st_pairs(lb_sim* sim, int on);

/* Rows per work item of the FV kernels (a launch-shape knob for tuning).
 * By default the height is chosen at the first step so that every item of a
 * launch is resident at once.  Any height >= 1 gives identical results
 * (fused steps take at least 2).  LB_EINVAL if rows < 1. */
int lb_set_fv_chunk(lb_sim* sim, int rows);

/* Fused steps (a launch-shape knob): for the semi-implicit + Heun scheme
 * with periodic x and FP32 arithmetic (not FP64 storage), one launch runs
 * the predictor (eq:semi) and the corrector (eq:semi-heun) of a step: each
 * block forms f~* on its strip and two cells beyond it and hands it to the
 * corrector through on-chip memory as FP32 offsets, with the collision base
 * f~n + C(f~n) of its cells, so a step reads f~n once and writes f~n+1 once
 * instead of moving five states.  With FP32 storage the results are
 * bit-identical to separate launches; with 16-bit storage f~* is not rounded
 * to the storage format (separate launches store it), one rounding fewer per
 * step.  on = 1 uses them wherever they apply, 0 never, -1 (the default)
 * where they measured faster on MI355X, which is everywhere they apply
 * (4096^2 with thermal populations: FP32 twice as fast, split BF16 +21%).
 * LB_EINVAL for other values. */
int lb_set_fv_fused(lb_sim* sim, int on);
/* The current setting (1, 0 or -1) in *on. */
int lb_get_fv_fused(const lb_sim* sim, int* on);

/* Number of bytes of device memory held by the handle. */
size_t lb_device_bytes(const lb_sim* sim);

/* ---- Serving: many simulations advanced by shared launches ------------
 *
 * A group holds up to max_sims FV semi-implicit + Heun simulations (same
 * storage format and thermal flag, any sizes, grids and parameters) and
 * advances all of them with one launch per step over the work items of
 * every member: a fused step (predictor and corrector, lb_set_fv_fused)
 * when every member takes fused steps alone, otherwise one predictor and
 * one corrector launch.  The launches are captured with the group's counter
 * updates (and the members' renewals of their thermal references,
 * lb_set_rebase) in a HIP graph of nsteps steps (re-captured only when the
 * membership or nsteps changes).  Each member carries its own remaining
 * step count and stops exactly there, so a member's state after its steps
 * is bit-identical to running it alone with lb_step in the same launch
 * shape: with fused group steps, alone with its settings; with separate
 * group launches (a member that does not take fused steps is present),
 * alone with lb_set_fv_fused(sim, 0), which for 16-bit storage differs from
 * fused steps by the rounding of f~* (FP32 and FP64: the same bits).
 * Members stay owned by
 * the caller.  While it is in a group, a member is advanced only by the
 * group: lb_step, lb_init, lb_set_grid, lb_set_state, lb_set_populations,
 * lb_rebase, lb_set_rebase, lb_set_fv_lanes, lb_set_fv_chunk and
 * lb_set_fv_fused on it return LB_ESTATE, and
 * so does adding it to a second group; reading it (lb_moments, lb_nusselt,
 * lb_get_state, ...) is allowed once the group's stream has been
 * synchronised (lb_group_sync or lb_group_remaining).
 * stream: hipStream_t to use, or NULL to create one. */
typedef struct lb_group lb_group;
int lb_group_create(int32_t max_sims, void* stream, lb_group** out);
void lb_group_destroy(lb_group* group);
/* Join with `steps` steps to do; *slot receives the member's slot.
 * LB_EINVAL for a non-Heun member, a storage/thermal mismatch or a second
 * add to the same group, LB_ESTATE without a state or for a member of
 * another group, LB_ENOMEM when all slots are taken.  Synchronises. */
int lb_group_add(lb_group* group, lb_sim* sim, int64_t steps, int32_t* slot);
/* Leave (finished or not); the slot becomes free and the simulation takes
 * its own automatic item height again.  Synchronises. */
int lb_group_remove(lb_group* group, int32_t slot);
/* Rows per work item of the members' launches: 0 (the default) chooses them
 * at each membership change from the members' strips and the number of
 * blocks the device holds at once (tall items when the members fill the
 * device many times over, short ones when few are left); rows >= 1 fixes
 * them.  Results do not depend on it.  Takes effect at the next
 * lb_group_step.  LB_EINVAL for a NULL group or rows < 0. */
int lb_group_set_chunk(lb_group* group, int32_t rows);
/* Enqueue nsteps group steps (asynchronous). */
int lb_group_step(lb_group* group, int64_t nsteps);
int lb_group_sync(lb_group* group);
/* Remaining steps of every slot (array of max_sims; 0 for free slots).
 * Synchronises. */
int lb_group_remaining(lb_group* group, int64_t* left);

/* Message of the last failing call on this thread ("" if none). */
const char* lb_last_error(void);

/* Streaming bandwidth of the current device, a reference ceiling for the
 * stage kernels' bandwidth (not part of the method).  Plain coalesced sweeps
 * of 16 bytes per lane over three device buffers of `bytes` each (rounded
 * down to 16 bytes, at least 16 MiB), allocated and freed by the call and
 * run on `stream` (hipStream_t or NULL); out[3] receives the best of three
 * launch shapes in GB/s for: 0 one read + one write per byte (a copy), 1 two
 * reads + one write, 2 two reads.  Synchronises the stream.  LB_EINVAL for a
 * NULL out or too small a size, LB_ENOMEM, LB_EDEVICE. */
int lb_stream_probe(size_t bytes, void* stream, double* out);

/* ======================================================================
 * Three dimensions: D3Q19, the lattice of the paper's own runs ("Boundary
 * conditions", last paragraph; sec. 5).  The same FV schemes (LB_FV_HEUN,
 * LB_FV_SEMI, LB_FV_EULER), QUICK along x, y and z, double reflection at
 * walls; gravity (Boussinesq a_z += beta_g (T - T0)) and the isothermal
 * walls (T_bottom at z_faces[0], T_top at z_faces[nz]) are along z, walls
 * normal to x or y are adiabatic for g.  Populations a = 0..18 have the
 * velocities
 *   (0,0,0) (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1)
 *   (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
 *   (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 * (weights 1/3, 1/18, 1/36).  Field arrays are [nz][ny][nx] (x fastest),
 * population arrays [19][nz][ny][nx].  Storage LB_F64 or LB_F32 (offsets
 * p - w rho_ref, g - w T_ref).  Each FV stage computes the brackets of its
 * input into a scratch buffer, then the flux divergence and the update
 * (see lb3_set_update).  Same error conventions as above.
 * ====================================================================== */
typedef struct lb3_params {
    int32_t nx, ny, nz;      /* cells, >= 4 each */
    int32_t scheme;          /* LB_FV_HEUN, LB_FV_SEMI or LB_FV_EULER */
    int32_t storage;         /* LB_F64 or LB_F32 */
    int32_t thermal;
    int32_t bc[3];           /* LB_PERIODIC or LB_WALL for x, y, z */
    double dt, tau, tau_g;   /* paper's tau, as in lb_params */
    double a[3];             /* constant acceleration */
    double beta_g, T0, T_bottom, T_top;
    double rho_ref, T_ref;   /* storage offsets for LB_F32 */
    void* stream;
} lb3_params;

typedef struct lb3_sim lb3_sim;

int lb3_create(const lb3_params* p, lb3_sim** out);
void lb3_destroy(lb3_sim* sim);
/* faces per axis, n+1 each, strictly increasing (copied); as lb_set_grid,
 * a failed later call leaves the previous grid in use */
int lb3_set_grid(lb3_sim* sim, const double* x_faces, int64_t n_xf, const double* y_faces, int64_t n_yf,
                 const double* z_faces, int64_t n_zf);
/* equilibrium start from host fields [nz][ny][nx]; T may be NULL unless thermal */
int lb3_init(lb3_sim* sim, const double* rho, const double* ux, const double* uy, const double* uz,
             const double* T);
int lb3_step(lb3_sim* sim, int64_t nsteps);
int lb3_sync(lb3_sim* sim);
/* rho, force-corrected u, T in double; any pointer may be NULL */
int lb3_moments(lb3_sim* sim, double* rho, double* ux, double* uy, double* uz, double* T);
/* decoded populations [19][nz][ny][nx] in double (g may be NULL) */
int lb3_get_populations(lb3_sim* sim, double* f, double* g);
/* out[8] as lb_diagnostics, the Nusselt numbers on the z walls */
int lb3_diagnostics(lb3_sim* sim, double* out);
/* Kernel of the flux + update half of each stage: 0 (default) tiles of
 * 32 x 4 x 4 cells whose brackets, with the halo cells their stencils
 * reach, are staged in LDS population by population; the kernel also
 * leaves the brackets of its output for the next stage in a second scratch
 * buffer, so the bracket kernel runs only after lb3_init.  1: one thread
 * per cell reading every stencil point from the scratch buffer, after a
 * bracket kernel in every stage.  Both compute the same operations in the
 * same order (bit-identical results).  LB_EINVAL for another kind. */
int lb3_set_update(lb3_sim* sim, int kind);
/* HIP-event timing of the stage passes: launches[2], ms[2] = (first pass, corrector) */
int lb3_set_timing(lb3_sim* sim, int on);
int lb3_kernel_times(lb3_sim* sim, int64_t* launches, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
