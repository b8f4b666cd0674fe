/*
 * FP64 CPU oracle for the finite-volume (FV) and streaming (ST) lattice
 * Boltzmann time steps of Shrestha, Mompean & Calzavarini (arXiv:1505.03271).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference the HIP
 * path is checked against.  It shares no code, header, table or helper with
 * the library under paper_1505_03271_amd/, and only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.
 *
 * Everything is double precision and follows the paper's notation:
 *   f~  ("ft")  redefined populations of the flow,  sec. 2.1 eq:ST
 *   g~  ("gt")  redefined thermal populations,       sec. 5 eq:LBg
 *   tau         the paper's relaxation time, nu = tau cs^2 (sec. 2)
 *   tau~        tau + dt/2                           (sec. 2.1)
 * Arrays are [q][ny][nx] with x fastest.  D2Q9 lattice (sec. 2.2, last
 * paragraph of "Boundary conditions": D3Q19 reduces to D2Q9 in 2D).
 *
 * Readings of points the paper leaves open (each one is listed in the design
 * notes of the repository):
 *  - f~eq is the standard second-order equilibrium of (rho, u) with u the
 *    force-corrected velocity of the "Force term" paragraph; eq:semi and
 *    eq:semi-heun are taken literally (the advected bracket carries +dt/2 F,
 *    the collision carries dt(1 - dt/(2 tau~)) F).
 *  - the Guo factor uses tau~ (as in eq:ST / eq:semi), not tau.
 *  - isothermal walls for g: ghost values are the anti-reflection
 *    phi_g,a(x_-k) = -phi_g,inv(a)(x_k) + 2 w_a T_w, the FV analogue of the
 *    anti-bounce-back rule; it makes the linear conductive profile an exact
 *    discrete steady state.  Walls normal to x are adiabatic for g (plain
 *    double reflection).
 *  - ST walls: half-way bounce-back for f, anti-bounce-back for g.
 *  - fixed-density boundaries ("Boundary conditions", second rule) are
 *    implemented for the flow populations of the FV schemes only; the paper
 *    gives no thermal rule for them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- D2Q9 lattice (textbook constants; the paper does not print them) ---- */
#define Q 9
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
/* inv(a): the population moving opposite to c_a ("Boundary conditions") */
static const int INV[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

enum { OB_FV_HEUN = 0, OB_FV_SEMI = 1, OB_FV_EULER = 2, OB_ST = 3 };

typedef struct {
    int32_t nx, ny;
    int32_t wall_x, wall_y; /* 0: periodic, 1: no-slip wall, 2: fixed density (FV, flow only) */
    int32_t thermal;        /* 1: double-population thermal model (sec. 5) */
    int32_t scheme;         /* OB_* */
    double dt;
    double tau, tau_g;      /* paper's tau: nu = tau cs^2, kappa = tau_g cs^2 */
    double ax, ay;          /* constant body acceleration */
    double beta_g, T0;      /* Boussinesq: a_y += beta g (T - T0) (sec. 5) */
    double T_bottom, T_top; /* isothermal wall temperatures on the y walls */
    double rho_lo, rho_hi;  /* fixed densities on the low / high face of a fixed-density axis */
} ob_params;

int ob_abi_version(void) { return 1; }

int ob_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (timing only; results do not
 * depend on it: every loop writes disjoint rows). */
void ob_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Grids (sec. 3, eq:grids).  faces[0..n]; cell centres are face midpoints.  */
/* ------------------------------------------------------------------------ */

void ob_grid_uniform(int n, double L, double* faces)
{
    for (int i = 0; i <= n; ++i) faces[i] = L * (double)i / (double)n;
}

/* hyperbolic-tangent stretching with factor s1 in (0,1) */
void ob_grid_tanh(int n, double L, double s1, double* faces)
{
    double a = atanh(s1);
    for (int i = 0; i <= n; ++i)
        faces[i] = 0.5 * L * (1.0 + tanh((2.0 * i / n - 1.0) * a) / s1);
    faces[0] = 0.0;
    faces[n] = L;
}

/* hyperbolic-sine stretching with factor s2 (n even) */
void ob_grid_sinh(int n, double L, double s2, double* faces)
{
    double A = 0.5 * L / sinh(0.5 * s2);
    for (int i = 0; i <= n; ++i) {
        if (2 * i <= n)
            faces[i] = A * sinh(s2 * i / n);
        else
            faces[i] = L - A * sinh(s2 * (n - i) / n);
    }
}

/* Centre of cell k on an axis, k may be a ghost index in [-2, n+1]:
 * periodic axes repeat with period L, wall axes mirror the first two fluid
 * centres about the wall face ("Boundary conditions"). */
static double centre(int n, const double* faces, int periodic, int k)
{
    double L = faces[n] - faces[0];
    if (k >= 0 && k < n) return 0.5 * (faces[k] + faces[k + 1]);
    if (periodic) {
        int m = ((k % n) + n) % n;
        double shift = (double)((k - m) / n) * L;
        return 0.5 * (faces[m] + faces[m + 1]) + shift;
    }
    if (k < 0) {
        int m = -k - 1; /* x_-1 mirrors x_1, x_-2 mirrors x_2 (0-based 0, 1) */
        return 2.0 * faces[0] - 0.5 * (faces[m] + faces[m + 1]);
    }
    int m = 2 * n - 1 - k;
    return 2.0 * faces[n] - 0.5 * (faces[m] + faces[m + 1]);
}

/* QUICK coefficients gamma_1..4 (sec. 2.2.3) for every face of one axis.
 * Face k (0..n) lies between cells k-1 and k.  Writing P = x_{k-1},
 * E = x_k, W = x_{k-2}, EE = x_{k+1} (the paper's x, x+, x-, x++) and xf
 * the face position, the upwind parabolas through (W,P,E) and (P,E,EE)
 * evaluated at xf give
 *   c.n > 0 : (1 - g1 + g2) f(P) + g1 f(E) - g2 f(W)
 *   c.n < 0 : (1 - g3 + g4) f(E) + g3 f(P) - g4 f(EE)
 * so g1, -g2 are the Lagrange weights of E and W on (W,P,E), and g3, -g4 the
 * weights of P and EE on (P,E,EE).  gam[4*k + 0..3] = g1, g2, g3, g4. */
void ob_quick_gammas(int n, const double* faces, int periodic, double* gam)
{
    for (int k = 0; k <= n; ++k) {
        double xf = faces[k];
        double Wp = centre(n, faces, periodic, k - 2);
        double P = centre(n, faces, periodic, k - 1);
        double E = centre(n, faces, periodic, k);
        double EE = centre(n, faces, periodic, k + 1);
        double g1 = (xf - Wp) * (xf - P) / ((E - Wp) * (E - P));
        double g2 = (xf - P) * (E - xf) / ((P - Wp) * (E - Wp));
        double g3 = (E - xf) * (EE - xf) / ((E - P) * (EE - P));
        double g4 = (xf - P) * (E - xf) / ((EE - P) * (EE - E));
        gam[4 * k + 0] = g1;
        gam[4 * k + 1] = g2;
        gam[4 * k + 2] = g3;
        gam[4 * k + 3] = g4;
    }
}

/* ------------------------------------------------------------------------ */
/* Local kinetic model: moments, equilibrium, Guo force (sec. 2, 2.1, 2.2.4, */
/* sec. 5).                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    double rho, ux, uy, T, ax, ay;
} ob_macro;

/* rho = sum f~, rho u = sum c f~ + dt/2 rho a, T = sum g~; the acceleration
 * includes the Boussinesq term, which depends on T only. */
static ob_macro macro_at(const ob_params* p, const double* ft, const double* gt,
                         size_t N, size_t c, double half_dt)
{
    ob_macro m;
    double rho = 0, jx = 0, jy = 0, T = 0;
    for (int a = 0; a < Q; ++a) {
        double v = ft[a * N + c];
        rho += v;
        jx += CX[a] * v;
        jy += CY[a] * v;
    }
    if (p->thermal)
        for (int a = 0; a < Q; ++a) T += gt[a * N + c];
    m.rho = rho;
    m.T = T;
    m.ax = p->ax;
    m.ay = p->ay + (p->thermal ? p->beta_g * (T - p->T0) : 0.0);
    m.ux = jx / rho + half_dt * m.ax;
    m.uy = jy / rho + half_dt * m.ay;
    return m;
}

static double feq_a(int a, double rho, double ux, double uy)
{
    double cu = CX[a] * ux + CY[a] * uy;
    double uu = ux * ux + uy * uy;
    return W[a] * rho * (1.0 + cu / CS2 + 0.5 * cu * cu / (CS2 * CS2) - 0.5 * uu / CS2);
}

/* eq:F2 (Guo et al.), without the (1 - dt/(2 tau~)) factor */
static double guo_a(int a, double rho, double ux, double uy, double ax, double ay)
{
    double cu = CX[a] * ux + CY[a] * uy;
    double t1x = (CX[a] - ux) / CS2 + cu * CX[a] / (CS2 * CS2);
    double t1y = (CY[a] - uy) / CS2 + cu * CY[a] / (CS2 * CS2);
    return W[a] * (t1x * ax + t1y * ay) * rho;
}

/* ------------------------------------------------------------------------ */
/* Initial state: populations at equilibrium with the prescribed rho, u, T. */
/* f~ at equilibrium is f_eq - dt/2 F (appendix A), so that the velocity    */
/* recovered by the "Force term" rule equals the prescribed u.               */
/* ------------------------------------------------------------------------ */

void ob_init(const ob_params* p, const double* rho, const double* ux,
             const double* uy, const double* T, double* ft, double* gt)
{
    size_t N = (size_t)p->nx * p->ny;
    double dt = (p->scheme == OB_ST) ? 1.0 : p->dt;
    double half = (p->scheme == OB_FV_EULER) ? 0.0 : 0.5 * dt;
    for (size_t c = 0; c < N; ++c) {
        double ax = p->ax;
        double ay = p->ay + (p->thermal ? p->beta_g * (T[c] - p->T0) : 0.0);
        for (int a = 0; a < Q; ++a) {
            double fe = feq_a(a, rho[c], ux[c], uy[c]);
            ft[a * N + c] = fe - half * guo_a(a, rho[c], ux[c], uy[c], ax, ay);
            if (p->thermal) gt[a * N + c] = T[c] / rho[c] * fe;
        }
    }
}

/* rho, force-corrected u, T of every cell (any output may be NULL) */
void ob_moments(const ob_params* p, const double* ft, const double* gt,
                double* rho, double* ux, double* uy, double* T)
{
    size_t N = (size_t)p->nx * p->ny;
    double dt = (p->scheme == OB_ST) ? 1.0 : p->dt;
    double half = (p->scheme == OB_FV_EULER) ? 0.0 : 0.5 * dt;
    for (size_t c = 0; c < N; ++c) {
        ob_macro m = macro_at(p, ft, gt, N, c, half);
        if (rho) rho[c] = m.rho;
        if (ux) ux[c] = m.ux;
        if (uy) uy[c] = m.uy;
        if (T) T[c] = m.T;
    }
}

/* ------------------------------------------------------------------------ */
/* FV step (sec. 2.2)                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    const ob_params* p;
    int nx, ny;
    size_t N;
    const double *xf, *yf;
    double *gx, *gy;     /* gammas per face, 4 per face */
    double *idx, *idy;   /* 1/dx_i, 1/dy_j (S_j / V on a rectilinear grid) */
} fv_ctx;

/* Advected field value of population a of species s (0: f, 1: g) at cell
 * index k along `axis`, the other index being `o`.  Ghost cells follow the
 * boundary rules, applied to the advected (physical) populations. */
static double node_value(const fv_ctx* C, const double* phi, int s, int a,
                         int axis, int k, int o)
{
    int n = axis == 0 ? C->nx : C->ny;
    int wall = axis == 0 ? C->p->wall_x : C->p->wall_y;
    int i, j;
    if (k >= 0 && k < n) {
        i = axis == 0 ? k : o;
        j = axis == 0 ? o : k;
        return phi[a * C->N + (size_t)j * C->nx + i];
    }
    if (!wall) {
        int m = ((k % n) + n) % n;
        i = axis == 0 ? m : o;
        j = axis == 0 ? o : m;
        return phi[a * C->N + (size_t)j * C->nx + i];
    }
    int m = k < 0 ? -k - 1 : 2 * n - 1 - k;
    i = axis == 0 ? m : o;
    j = axis == 0 ? o : m;
    if (wall == 2) {
        /* fixed density rho_S on the boundary face: the ghost density is the
         * linear extrapolation through (x_S, rho_S) and (x_k, rho(x_k)) to
         * the mirror point x_-k, i.e. 2 rho_S - rho(x_k), and the ghost
         * populations are the mirror cell's rescaled by rho(x_-k)/rho(x_k) */
        double rhoS = k < 0 ? C->p->rho_lo : C->p->rho_hi;
        double rk = 0.0;
        for (int b = 0; b < Q; ++b) rk += phi[b * C->N + (size_t)j * C->nx + i];
        double rg = 2.0 * rhoS - rk;
        return rg / rk * phi[a * C->N + (size_t)j * C->nx + i];
    }
    /* double reflection: f_a(x_-k) = f_inv(a)(x_k) */
    double v = phi[INV[a] * C->N + (size_t)j * C->nx + i];
    if (s == 1 && axis == 1) {
        /* isothermal y walls: anti-reflection about the wall temperature */
        double Tw = k < 0 ? C->p->T_bottom : C->p->T_top;
        v = -v + 2.0 * W[a] * Tw;
    }
    return v;
}

/* QUICK face value of population a on the face between cells k and k+1 of
 * `axis` (k in [-1, n-1]); periodic axes map k = -1 to the last face. */
static double face_value(const fv_ctx* C, const double* phi, int s, int a,
                         int axis, int k, int o)
{
    int n = axis == 0 ? C->nx : C->ny;
    int wall = axis == 0 ? C->p->wall_x : C->p->wall_y;
    if (!wall && k < 0) k += n;
    int cn = axis == 0 ? CX[a] : CY[a];
    const double* gm = (axis == 0 ? C->gx : C->gy) + 4 * (k + 1);
    double P = node_value(C, phi, s, a, axis, k, o);
    double E = node_value(C, phi, s, a, axis, k + 1, o);
    if (cn > 0) {
        double Wv = node_value(C, phi, s, a, axis, k - 1, o);
        return (1.0 - gm[0] + gm[1]) * P + gm[0] * E - gm[1] * Wv;
    } else {
        double EE = node_value(C, phi, s, a, axis, k + 2, o);
        return (1.0 - gm[2] + gm[3]) * E + gm[2] * P - gm[3] * EE;
    }
}

/* D_a = (S_j / V) c_a . n_j [phi_a]_j : the net outflow of eq:fv */
static void flux(const fv_ctx* C, const double* phi, int s, double* D)
{
    int nx = C->nx, ny = C->ny;
    size_t N = C->N;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            D[c] = 0.0; /* rest population: no flux */
            for (int a = 1; a < Q; ++a) {
                double d = 0.0;
                if (CX[a] != 0)
                    d += CX[a] * (face_value(C, phi, s, a, 0, i, j) -
                                  face_value(C, phi, s, a, 0, i - 1, j)) * C->idx[i];
                if (CY[a] != 0)
                    d += CY[a] * (face_value(C, phi, s, a, 1, j, i) -
                                  face_value(C, phi, s, a, 1, j - 1, i)) * C->idy[j];
                D[a * N + c] = d;
            }
        }
}

/* Reading of the advected bracket's force term (an oracle-only switch, to
 * measure what the choice moves): 0, the literal eq:semi / eq:semi-heun
 * (+dt/2 F, the default); 1, the physical distribution of the Crank-Nicolson
 * transform, whose force term is dt/2 (1 - dt/(2 tau~)) F, i.e. dt^2/(4 tau~)
 * F less. */
static int g_bracket_alt = 0;
void ob_set_bracket(int alt) { g_bracket_alt = alt ? 1 : 0; }

/* Local part of one semi-implicit stage (eq:semi): the advected bracket
 * phi = f~ + dt/(2 tau~)(f~eq - f~) + dt/2 F and the collision + force
 * increment Cf = dt/tau~ (f~eq - f~) + dt (1 - dt/(2 tau~)) F, and the same
 * for g~ with g~eq = (T/rho) f~eq and no source (eq:LBg).  For the explicit
 * Euler variant (eq:euler) phi = f and C = dt/tau (feq - f) + dt F. */
static void stage(const fv_ctx* C, const double* ft, const double* gt,
                  double* phf, double* Cf, double* phg, double* Cg)
{
    const ob_params* p = C->p;
    size_t N = C->N;
    double dt = p->dt;
    int euler = p->scheme == OB_FV_EULER;
    double tt = euler ? p->tau : p->tau + 0.5 * dt;
    double ttg = euler ? p->tau_g : p->tau_g + 0.5 * dt;
    double half = euler ? 0.0 : 0.5 * dt;
#pragma omp parallel for schedule(static)
    for (long long cc = 0; cc < (long long)N; ++cc) {
        size_t c = (size_t)cc;
        ob_macro m = macro_at(p, ft, gt, N, c, half);
        for (int a = 0; a < Q; ++a) {
            double f = ft[a * N + c];
            double fe = feq_a(a, m.rho, m.ux, m.uy);
            double F = guo_a(a, m.rho, m.ux, m.uy, m.ax, m.ay);
            if (euler) {
                phf[a * N + c] = f;
                if (Cf) Cf[a * N + c] = dt / tt * (fe - f) + dt * F;
            } else {
                double kf = g_bracket_alt ? 0.5 * dt * (1.0 - dt / (2.0 * tt)) : 0.5 * dt;
                phf[a * N + c] = f + dt / (2.0 * tt) * (fe - f) + kf * F;
                if (Cf) Cf[a * N + c] = dt / tt * (fe - f) + dt * (1.0 - dt / (2.0 * tt)) * F;
            }
            if (p->thermal) {
                double g = gt[a * N + c];
                double ge = m.T / m.rho * fe;
                if (euler)
                    phg[a * N + c] = g;
                else
                    phg[a * N + c] = g + dt / (2.0 * ttg) * (ge - g);
                if (Cg) Cg[a * N + c] = dt / ttg * (ge - g);
            }
        }
    }
}

static int fv_setup(fv_ctx* C, const ob_params* p, const double* xf, const double* yf)
{
    C->p = p;
    C->nx = p->nx;
    C->ny = p->ny;
    C->N = (size_t)p->nx * p->ny;
    C->xf = xf;
    C->yf = yf;
    C->gx = malloc(sizeof(double) * 4 * (p->nx + 1));
    C->gy = malloc(sizeof(double) * 4 * (p->ny + 1));
    C->idx = malloc(sizeof(double) * p->nx);
    C->idy = malloc(sizeof(double) * p->ny);
    if (!C->gx || !C->gy || !C->idx || !C->idy) return -1;
    ob_quick_gammas(p->nx, xf, !p->wall_x, C->gx);
    ob_quick_gammas(p->ny, yf, !p->wall_y, C->gy);
    for (int i = 0; i < p->nx; ++i) C->idx[i] = 1.0 / (xf[i + 1] - xf[i]);
    for (int j = 0; j < p->ny; ++j) C->idy[j] = 1.0 / (yf[j + 1] - yf[j]);
    return 0;
}

static void fv_free(fv_ctx* C)
{
    free(C->gx);
    free(C->gy);
    free(C->idx);
    free(C->idy);
}

/* Advance (ft, gt) in place by nsteps FV steps of the chosen scheme:
 *   Euler   eq:euler
 *   semi    eq:semi                      f~(t+dt) = f~ - dt D(phi) + C
 *   Heun    eq:semi-heun  f~* = f~ - dt D(phi) + C,
 *           f~(t+dt) = f~ - dt/2 (D(phi) + D(phi*)) + C
 * where phi* and F* are evaluated from f~* (and g~*). */
int ob_fv_run(const ob_params* p, const double* xf, const double* yf,
              double* ft, double* gt, long long nsteps)
{
    fv_ctx C;
    if (p->nx < 1 || p->ny < 1 || p->scheme == OB_ST) return -1;
    if (p->thermal && (p->wall_x == 2 || p->wall_y == 2)) return -1;
    if (fv_setup(&C, p, xf, yf)) return -2;
    size_t N = C.N, QN = Q * N;
    int th = p->thermal;
    double* buf = malloc(sizeof(double) * QN * (th ? 10 : 5));
    if (!buf) {
        fv_free(&C);
        return -2;
    }
    double *phf = buf, *Cf = buf + QN, *Df = buf + 2 * QN, *fs = buf + 3 * QN,
           *Ds = buf + 4 * QN;
    double *phg = th ? buf + 5 * QN : NULL, *Cg = th ? buf + 6 * QN : NULL,
           *Dg = th ? buf + 7 * QN : NULL, *gs = th ? buf + 8 * QN : NULL,
           *Dgs = th ? buf + 9 * QN : NULL;
    double dt = p->dt;
    for (long long n = 0; n < nsteps; ++n) {
        stage(&C, ft, gt, phf, Cf, phg, Cg);
        flux(&C, phf, 0, Df);
        if (th) flux(&C, phg, 1, Dg);
        if (p->scheme != OB_FV_HEUN) {
            for (size_t k = 0; k < QN; ++k) ft[k] += -dt * Df[k] + Cf[k];
            if (th)
                for (size_t k = 0; k < QN; ++k) gt[k] += -dt * Dg[k] + Cg[k];
            continue;
        }
        /* predictor (eq:semi) */
        for (size_t k = 0; k < QN; ++k) fs[k] = ft[k] - dt * Df[k] + Cf[k];
        if (th)
            for (size_t k = 0; k < QN; ++k) gs[k] = gt[k] - dt * Dg[k] + Cg[k];
        /* corrector (eq:semi-heun): advected bracket of the predicted state */
        stage(&C, fs, gs, phf, NULL, phg, NULL);
        flux(&C, phf, 0, Ds);
        if (th) flux(&C, phg, 1, Dgs);
        for (size_t k = 0; k < QN; ++k) ft[k] += -0.5 * dt * (Df[k] + Ds[k]) + Cf[k];
        if (th)
            for (size_t k = 0; k < QN; ++k) gt[k] += -0.5 * dt * (Dg[k] + Dgs[k]) + Cg[k];
    }
    free(buf);
    fv_free(&C);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ST step (sec. 2.1, eq:ST) with dt = dx = 1                                */
/* ------------------------------------------------------------------------ */

/* Destination of population a leaving cell (i, j): the neighbour x + c_a, or,
 * when that neighbour lies beyond a wall, the slot inv(a) of the same cell
 * (half-way bounce-back).  Returns 1 when the move hit a wall; *hit_top tells
 * which y wall was hit (for the thermal rule). */
static int st_dest(const ob_params* p, int a, int i, int j, int* di, int* dj,
                   int* da, int* ywall)
{
    int ti = i + CX[a], tj = j + CY[a];
    int hit = 0;
    *ywall = 0;
    if (tj < 0 || tj >= p->ny) {
        if (p->wall_y) {
            hit = 1;
            *ywall = tj < 0 ? -1 : 1;
        } else
            tj = (tj + p->ny) % p->ny;
    }
    if (ti < 0 || ti >= p->nx) {
        if (p->wall_x)
            hit = 1;
        else
            ti = (ti + p->nx) % p->nx;
    }
    if (hit) {
        *di = i;
        *dj = j;
        *da = INV[a];
    } else {
        *di = ti;
        *dj = tj;
        *da = a;
    }
    return hit;
}

/* Post-collision value of eq:ST's right-hand side, then streaming. */
int ob_st_run(const ob_params* p, double* ft, double* gt, long long nsteps)
{
    if (p->wall_x == 2 || p->wall_y == 2) return -1; /* fixed density: FV only */
    size_t N = (size_t)p->nx * p->ny, QN = Q * N;
    int th = p->thermal;
    double* nf = malloc(sizeof(double) * QN);
    double* ng = th ? malloc(sizeof(double) * QN) : NULL;
    if (!nf || (th && !ng)) {
        free(nf);
        free(ng);
        return -2;
    }
    const double dt = 1.0;
    double tt = p->tau + 0.5 * dt, ttg = p->tau_g + 0.5 * dt;
    for (long long n = 0; n < nsteps; ++n) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                size_t c = (size_t)j * p->nx + i;
                ob_macro m = macro_at(p, ft, gt, N, c, 0.5 * dt);
                for (int a = 0; a < Q; ++a) {
                    double f = ft[a * N + c];
                    double fe = feq_a(a, m.rho, m.ux, m.uy);
                    double F = guo_a(a, m.rho, m.ux, m.uy, m.ax, m.ay);
                    double fpost = f + dt / tt * (fe - f) + dt * (1.0 - dt / (2.0 * tt)) * F;
                    int di, dj, da, yw;
                    st_dest(p, a, i, j, &di, &dj, &da, &yw);
                    nf[da * N + (size_t)dj * p->nx + di] = fpost;
                    if (th) {
                        double g = gt[a * N + c];
                        double ge = m.T / m.rho * fe;
                        double gpost = g + dt / ttg * (ge - g);
                        if (yw != 0) /* anti-bounce-back at isothermal walls */
                            gpost = -gpost + 2.0 * W[a] * (yw < 0 ? p->T_bottom : p->T_top);
                        ng[da * N + (size_t)dj * p->nx + di] = gpost;
                    }
                }
            }
        memcpy(ft, nf, sizeof(double) * QN);
        if (th) memcpy(gt, ng, sizeof(double) * QN);
    }
    free(nf);
    free(ng);
    return 0;
}

/* Streaming alone, as a permutation of storage slots: for every destination
 * slot (a, j, i) the source slot it receives, both as a*N + j*nx + i.  The
 * thermal populations follow the same map. */
void ob_st_stream_sources(const ob_params* p, int64_t* src)
{
    size_t N = (size_t)p->nx * p->ny;
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i)
            for (int a = 0; a < Q; ++a) {
                int di, dj, da, yw;
                st_dest(p, a, i, j, &di, &dj, &da, &yw);
                src[da * N + (size_t)dj * p->nx + di] = (int64_t)(a * N + (size_t)j * p->nx + i);
            }
}

/* ------------------------------------------------------------------------ */
/* Diagnostics (sec. 3.1 kinetic energy; sec. 5 Nusselt number)              */
/* out[0] mass      sum V rho                                                */
/* out[1] kinetic   sum V rho |u|^2 / 2                                      */
/* out[2] thermal   sum V T                                                  */
/* out[3] Nu bottom  -H dT/dy(0) / dT, wall-averaged, 2nd-order one-sided    */
/* out[4] Nu top     -H dT/dy(H) / dT, same                                  */
/* out[5] Nu volume  1 + H <u_y T>_V / (kappa dT)                            */
/* out[6] volume    sum V                                                    */
/* out[7] 1 if any population is not finite                                  */
/* ------------------------------------------------------------------------ */

/* derivative at x0 of the parabola through (x0,f0), (x1,f1), (x2,f2) */
static double d_parabola(double x0, double f0, double x1, double f1, double x2, double f2)
{
    return f0 * ((x0 - x1) + (x0 - x2)) / ((x0 - x1) * (x0 - x2)) +
           f1 * (x0 - x2) / ((x1 - x0) * (x1 - x2)) +
           f2 * (x0 - x1) / ((x2 - x0) * (x2 - x1));
}

void ob_diagnostics(const ob_params* p, const double* xf, const double* yf,
                    const double* ft, const double* gt, double* out)
{
    int nx = p->nx, ny = p->ny;
    size_t N = (size_t)nx * ny;
    double dt = (p->scheme == OB_ST) ? 1.0 : p->dt;
    double half = (p->scheme == OB_FV_EULER) ? 0.0 : 0.5 * dt;
    double M = 0, Ek = 0, Et = 0, uT = 0, V = 0;
    int bad = 0;
    double* T = malloc(sizeof(double) * N);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            ob_macro m = macro_at(p, ft, gt, N, c, half);
            double v = (xf[i + 1] - xf[i]) * (yf[j + 1] - yf[j]);
            M += v * m.rho;
            Ek += v * 0.5 * m.rho * (m.ux * m.ux + m.uy * m.uy);
            Et += v * m.T;
            uT += v * m.uy * m.T;
            V += v;
            T[c] = m.T;
            for (int a = 0; a < Q; ++a) {
                if (!isfinite(ft[a * N + c])) bad = 1;
                if (p->thermal && !isfinite(gt[a * N + c])) bad = 1;
            }
        }
    double nub = 0, nut = 0, nuv = 0;
    if (p->thermal && p->wall_y && ny >= 2) {
        double H = yf[ny] - yf[0];
        double dT = p->T_bottom - p->T_top;
        double kappa = p->tau_g * CS2;
        double y0 = 0.5 * (yf[0] + yf[1]), y1 = 0.5 * (yf[1] + yf[2]);
        double z0 = 0.5 * (yf[ny - 1] + yf[ny]), z1 = 0.5 * (yf[ny - 2] + yf[ny - 1]);
        double Lx = xf[nx] - xf[0];
        for (int i = 0; i < nx; ++i) {
            double w = (xf[i + 1] - xf[i]) / Lx;
            double gb = d_parabola(yf[0], p->T_bottom, y0, T[i], y1, T[(size_t)nx + i]);
            double gtp = d_parabola(yf[ny], p->T_top, z0, T[(size_t)(ny - 1) * nx + i], z1,
                                    T[(size_t)(ny - 2) * nx + i]);
            nub += w * (-gb * H / dT);
            nut += w * (-gtp * H / dT);
        }
        nuv = 1.0 + H * (uT / V) / (kappa * dT);
    }
    free(T);
    out[0] = M;
    out[1] = Ek;
    out[2] = Et;
    out[3] = nub;
    out[4] = nut;
    out[5] = nuv;
    out[6] = V;
    out[7] = bad;
}

/* ======================================================================== */
/* Three dimensions: D3Q19 (the lattice of the paper's own runs, "Boundary   */
/* conditions", last paragraph; sec. 5).  Same scheme, face by face along    */
/* x, y and z; gravity and the isothermal walls are along z.                 */
/* ======================================================================== */

#define Q3 19
/* rest, 6 axis velocities, 12 edge velocities; opposite pairs adjacent */
static const int C3[Q3][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double w3(int a)
{
    int s = abs(C3[a][0]) + abs(C3[a][1]) + abs(C3[a][2]);
    return s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

static int inv3(int a)
{
    for (int b = 0; b < Q3; ++b)
        if (C3[b][0] == -C3[a][0] && C3[b][1] == -C3[a][1] && C3[b][2] == -C3[a][2]) return b;
    return -1;
}

typedef struct {
    int32_t nx, ny, nz;
    int32_t wall[3];        /* per axis: 0 periodic, 1 no-slip wall */
    int32_t thermal, scheme;
    double dt, tau, tau_g;
    double a0[3];           /* constant acceleration */
    double beta_g, T0;      /* a_z += beta g (T - T0) */
    double T_bottom, T_top; /* isothermal z walls */
} ob3_params;

typedef struct {
    double rho, u[3], T, a[3];
} ob3_macro;

static ob3_macro macro3(const ob3_params* p, const double* ft, const double* gt, size_t N, size_t c,
                        double half)
{
    ob3_macro m;
    double rho = 0, j[3] = {0, 0, 0}, T = 0;
    for (int a = 0; a < Q3; ++a) {
        double v = ft[a * N + c];
        rho += v;
        for (int d = 0; d < 3; ++d) j[d] += C3[a][d] * v;
    }
    if (p->thermal)
        for (int a = 0; a < Q3; ++a) T += gt[a * N + c];
    m.rho = rho;
    m.T = T;
    for (int d = 0; d < 3; ++d) m.a[d] = p->a0[d];
    if (p->thermal) m.a[2] += p->beta_g * (T - p->T0);
    for (int d = 0; d < 3; ++d) m.u[d] = j[d] / rho + half * m.a[d];
    return m;
}

static double feq3(int a, double rho, const double* u)
{
    double cu = 0, uu = 0;
    for (int d = 0; d < 3; ++d) {
        cu += C3[a][d] * u[d];
        uu += u[d] * u[d];
    }
    return w3(a) * rho * (1.0 + cu / CS2 + 0.5 * cu * cu / (CS2 * CS2) - 0.5 * uu / CS2);
}

static double guo3(int a, double rho, const double* u, const double* acc)
{
    double cu = 0, s = 0;
    for (int d = 0; d < 3; ++d) cu += C3[a][d] * u[d];
    for (int d = 0; d < 3; ++d) s += ((C3[a][d] - u[d]) / CS2 + cu * C3[a][d] / (CS2 * CS2)) * acc[d];
    return w3(a) * s * rho;
}

int ob3_abi_version(void) { return 1; }

void ob3_init(const ob3_params* p, const double* rho, const double* ux, const double* uy, const double* uz,
              const double* T, double* ft, double* gt)
{
    size_t N = (size_t)p->nx * p->ny * p->nz;
    double half = p->scheme == OB_FV_EULER ? 0.0 : 0.5 * p->dt;
    for (size_t c = 0; c < N; ++c) {
        double u[3] = {ux[c], uy[c], uz[c]};
        double acc[3] = {p->a0[0], p->a0[1], p->a0[2] + (p->thermal ? p->beta_g * (T[c] - p->T0) : 0.0)};
        for (int a = 0; a < Q3; ++a) {
            double fe = feq3(a, rho[c], u);
            ft[a * N + c] = fe - half * guo3(a, rho[c], u, acc);
            if (p->thermal) gt[a * N + c] = T[c] / rho[c] * fe;
        }
    }
}

void ob3_moments(const ob3_params* p, const double* ft, const double* gt, double* rho, double* ux,
                 double* uy, double* uz, double* T)
{
    size_t N = (size_t)p->nx * p->ny * p->nz;
    double half = p->scheme == OB_FV_EULER ? 0.0 : 0.5 * p->dt;
    for (size_t c = 0; c < N; ++c) {
        ob3_macro m = macro3(p, ft, gt, N, c, half);
        if (rho) rho[c] = m.rho;
        if (ux) ux[c] = m.u[0];
        if (uy) uy[c] = m.u[1];
        if (uz) uz[c] = m.u[2];
        if (T) T[c] = m.T;
    }
}

typedef struct {
    const ob3_params* p;
    int n[3];
    size_t N;
    const double* faces[3];
    double* gam[3];  /* QUICK gammas per axis, 4 per face */
    double* inv[3];  /* 1 / cell width per axis */
} fv3_ctx;

/* advected value of population a (species s) at index k along `axis`, the
 * cell's other two indices taken from (i, j, l) */
static double node3(const fv3_ctx* C, const double* phi, int s, int a, int axis, int k, int i, int j, int l)
{
    int n = C->n[axis];
    int idx[3] = {i, j, l};
    int wall = C->p->wall[axis];
    int b = a;
    double sgn = 1.0, add = 0.0;
    if (k >= 0 && k < n) {
        idx[axis] = k;
    } else if (!wall) {
        idx[axis] = ((k % n) + n) % n;
    } else {
        /* double reflection; isothermal anti-reflection for g on z walls */
        idx[axis] = k < 0 ? -k - 1 : 2 * n - 1 - k;
        b = inv3(a);
        if (s == 1 && axis == 2) {
            sgn = -1.0;
            add = 2.0 * w3(a) * (k < 0 ? C->p->T_bottom : C->p->T_top);
        }
    }
    size_t c = ((size_t)idx[2] * C->n[1] + idx[1]) * C->n[0] + idx[0];
    return sgn * phi[b * C->N + c] + add;
}

static double face3(const fv3_ctx* C, const double* phi, int s, int a, int axis, int k, int i, int j, int l)
{
    int n = C->n[axis];
    if (!C->p->wall[axis] && k < 0) k += n;
    const double* gm = C->gam[axis] + 4 * (k + 1);
    double P = node3(C, phi, s, a, axis, k, i, j, l);
    double E = node3(C, phi, s, a, axis, k + 1, i, j, l);
    if (C3[a][axis] > 0) {
        double Wv = node3(C, phi, s, a, axis, k - 1, i, j, l);
        return (1.0 - gm[0] + gm[1]) * P + gm[0] * E - gm[1] * Wv;
    }
    double EE = node3(C, phi, s, a, axis, k + 2, i, j, l);
    return (1.0 - gm[2] + gm[3]) * E + gm[2] * P - gm[3] * EE;
}

static void flux3(const fv3_ctx* C, const double* phi, int s, double* D)
{
    int nx = C->n[0], ny = C->n[1], nz = C->n[2];
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = ((size_t)l * ny + j) * nx + i;
                int pos[3] = {i, j, l};
                D[c] = 0.0;
                for (int a = 1; a < Q3; ++a) {
                    double d = 0.0;
                    for (int ax = 0; ax < 3; ++ax)
                        if (C3[a][ax] != 0)
                            d += C3[a][ax] * (face3(C, phi, s, a, ax, pos[ax], i, j, l) -
                                              face3(C, phi, s, a, ax, pos[ax] - 1, i, j, l)) * C->inv[ax][pos[ax]];
                    D[a * C->N + c] = d;
                }
            }
}

static void stage3(const fv3_ctx* C, const double* ft, const double* gt, double* phf, double* Cf, double* phg,
                   double* Cg)
{
    const ob3_params* p = C->p;
    size_t N = C->N;
    double dt = p->dt;
    int euler = p->scheme == OB_FV_EULER;
    double tt = euler ? p->tau : p->tau + 0.5 * dt;
    double ttg = euler ? p->tau_g : p->tau_g + 0.5 * dt;
    double half = euler ? 0.0 : 0.5 * dt;
#pragma omp parallel for schedule(static)
    for (long long cc = 0; cc < (long long)N; ++cc) {
        size_t c = (size_t)cc;
        ob3_macro m = macro3(p, ft, gt, N, c, half);
        for (int a = 0; a < Q3; ++a) {
            double f = ft[a * N + c];
            double fe = feq3(a, m.rho, m.u);
            double F = guo3(a, m.rho, m.u, m.a);
            if (euler) {
                phf[a * N + c] = f;
                if (Cf) Cf[a * N + c] = dt / tt * (fe - f) + dt * F;
            } else {
                double kf = g_bracket_alt ? 0.5 * dt * (1.0 - dt / (2.0 * tt)) : 0.5 * dt;
                phf[a * N + c] = f + dt / (2.0 * tt) * (fe - f) + kf * F;
                if (Cf) Cf[a * N + c] = dt / tt * (fe - f) + dt * (1.0 - dt / (2.0 * tt)) * F;
            }
            if (p->thermal) {
                double g = gt[a * N + c];
                double ge = m.T / m.rho * fe;
                phg[a * N + c] = euler ? g : g + dt / (2.0 * ttg) * (ge - g);
                if (Cg) Cg[a * N + c] = dt / ttg * (ge - g);
            }
        }
    }
}

int ob3_fv_run(const ob3_params* p, const double* xf, const double* yf, const double* zf, double* ft,
               double* gt, long long nsteps)
{
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->scheme == OB_ST) return -1;
    fv3_ctx C;
    C.p = p;
    C.n[0] = p->nx;
    C.n[1] = p->ny;
    C.n[2] = p->nz;
    C.N = (size_t)p->nx * p->ny * p->nz;
    C.faces[0] = xf;
    C.faces[1] = yf;
    C.faces[2] = zf;
    int ok = 1;
    for (int d = 0; d < 3; ++d) {
        C.gam[d] = malloc(sizeof(double) * 4 * (C.n[d] + 1));
        C.inv[d] = malloc(sizeof(double) * C.n[d]);
        if (!C.gam[d] || !C.inv[d]) ok = 0;
    }
    size_t N = C.N, QN = Q3 * N;
    int th = p->thermal;
    double* buf = ok ? malloc(sizeof(double) * QN * (th ? 10 : 5)) : NULL;
    if (!buf) {
        for (int d = 0; d < 3; ++d) {
            free(C.gam[d]);
            free(C.inv[d]);
        }
        return -2;
    }
    for (int d = 0; d < 3; ++d) {
        ob_quick_gammas(C.n[d], C.faces[d], !p->wall[d], C.gam[d]);
        for (int k = 0; k < C.n[d]; ++k) C.inv[d][k] = 1.0 / (C.faces[d][k + 1] - C.faces[d][k]);
    }
    double *phf = buf, *Cf = buf + QN, *Df = buf + 2 * QN, *fs = buf + 3 * QN, *Ds = buf + 4 * QN;
    double *phg = th ? buf + 5 * QN : NULL, *Cg = th ? buf + 6 * QN : NULL, *Dg = th ? buf + 7 * QN : NULL,
           *gs = th ? buf + 8 * QN : NULL, *Dgs = th ? buf + 9 * QN : NULL;
    double dt = p->dt;
    for (long long n = 0; n < nsteps; ++n) {
        stage3(&C, ft, gt, phf, Cf, phg, Cg);
        flux3(&C, phf, 0, Df);
        if (th) flux3(&C, phg, 1, Dg);
        if (p->scheme != OB_FV_HEUN) {
            for (size_t k = 0; k < QN; ++k) ft[k] += -dt * Df[k] + Cf[k];
            if (th)
                for (size_t k = 0; k < QN; ++k) gt[k] += -dt * Dg[k] + Cg[k];
            continue;
        }
        for (size_t k = 0; k < QN; ++k) fs[k] = ft[k] - dt * Df[k] + Cf[k];
        if (th)
            for (size_t k = 0; k < QN; ++k) gs[k] = gt[k] - dt * Dg[k] + Cg[k];
        stage3(&C, fs, gs, phf, NULL, phg, NULL);
        flux3(&C, phf, 0, Ds);
        if (th) flux3(&C, phg, 1, Dgs);
        for (size_t k = 0; k < QN; ++k) ft[k] += -0.5 * dt * (Df[k] + Ds[k]) + Cf[k];
        if (th)
            for (size_t k = 0; k < QN; ++k) gt[k] += -0.5 * dt * (Dg[k] + Dgs[k]) + Cg[k];
    }
    free(buf);
    for (int d = 0; d < 3; ++d) {
        free(C.gam[d]);
        free(C.inv[d]);
    }
    return 0;
}

/* out[8] as ob_diagnostics, with the Nusselt numbers on the z walls
 * (horizontal averages over x and y, weighted by the cell areas) */
void ob3_diagnostics(const ob3_params* p, const double* xf, const double* yf, const double* zf,
                     const double* ft, const double* gt, double* out)
{
    int nx = p->nx, ny = p->ny, nz = p->nz;
    size_t N = (size_t)nx * ny * nz, A = (size_t)nx * ny;
    double half = p->scheme == OB_FV_EULER ? 0.0 : 0.5 * p->dt;
    double M = 0, Ek = 0, Et = 0, uT = 0, V = 0;
    int bad = 0;
    double* T = malloc(sizeof(double) * N);
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = ((size_t)l * ny + j) * nx + i;
                ob3_macro m = macro3(p, ft, gt, N, c, half);
                double v = (xf[i + 1] - xf[i]) * (yf[j + 1] - yf[j]) * (zf[l + 1] - zf[l]);
                M += v * m.rho;
                Ek += v * 0.5 * m.rho * (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2]);
                Et += v * m.T;
                uT += v * m.u[2] * m.T;
                V += v;
                T[c] = m.T;
                for (int a = 0; a < Q3; ++a) {
                    if (!isfinite(ft[a * N + c])) bad = 1;
                    if (p->thermal && !isfinite(gt[a * N + c])) bad = 1;
                }
            }
    double nub = 0, nut = 0, nuv = 0;
    if (p->thermal && p->wall[2] && nz >= 2) {
        double H = zf[nz] - zf[0], dT = p->T_bottom - p->T_top, kappa = p->tau_g * CS2;
        double z0 = 0.5 * (zf[0] + zf[1]), z1 = 0.5 * (zf[1] + zf[2]);
        double t0 = 0.5 * (zf[nz - 1] + zf[nz]), t1 = 0.5 * (zf[nz - 2] + zf[nz - 1]);
        double Area = (xf[nx] - xf[0]) * (yf[ny] - yf[0]);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = (size_t)j * nx + i;
                double w = (xf[i + 1] - xf[i]) * (yf[j + 1] - yf[j]) / Area;
                double gb = d_parabola(zf[0], p->T_bottom, z0, T[c], z1, T[A + c]);
                double gtp = d_parabola(zf[nz], p->T_top, t0, T[(size_t)(nz - 1) * A + c], t1,
                                        T[(size_t)(nz - 2) * A + c]);
                nub += w * (-gb * H / dT);
                nut += w * (-gtp * H / dT);
            }
        nuv = 1.0 + H * (uT / V) / (kappa * dT);
    }
    free(T);
    out[0] = M;
    out[1] = Ek;
    out[2] = Et;
    out[3] = nub;
    out[4] = nut;
    out[5] = nuv;
    out[6] = V;
    out[7] = bad;
}
