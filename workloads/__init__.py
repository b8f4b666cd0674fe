"""Seeded synthetic workloads for the FV-LB / ST-LB time step.

This module defines inputs only: grid face coordinates, initial macroscopic
fields (rho, u, T), physical parameters and the serving request trace.  It
holds none of the method's arithmetic (no equilibrium, no collision, no flux)
and is shared by the oracle tests and the HIP-path tests and benchmark, so
both sides always start from the same numbers.

Random numbers come from NumPy's PCG64 with seed ``150503271 + index``.

Configurations (lattice units throughout):
  tgv64      Taylor-Green vortex, 64x64 periodic, u0 = 0.01, nu = 0.1
  channel    body-force channel 256 (periodic) x 512 (walls), tanh(2.0) in y,
             nu = 1/30, Re_bulk = 1000, uniform +-1e-3 velocity noise
  rb1024     Rayleigh-Benard Ra = 1e8, Pr = 1, aspect 1, 1024^2, tanh(2.0) in y
  serving    Poisson request trace of Rayleigh-Benard runs (see serving_trace)
  rb4096     Rayleigh-Benard Ra = 1e10, Pr = 1, 4096^2, tanh(2.5) in y
"""
import math

import numpy as np

SEED_BASE = 150503271
CS2 = 1.0 / 3.0


def rng(index):
    return np.random.Generator(np.random.PCG64(SEED_BASE + index))


# ---------------------------------------------------------------- grids ----

def faces_uniform(n, L):
    return L * np.arange(n + 1, dtype=np.float64) / n


def faces_tanh(n, L, stretch):
    """Hyperbolic-tangent wall refinement (sec. 3, eq:grids) with the paper's
    factor s1 = tanh(stretch); stretch 2.0 gives a min/max cell ratio of 0.071."""
    s1 = math.tanh(stretch)
    i = np.arange(n + 1, dtype=np.float64)
    xi = 0.5 * L * (1.0 + np.tanh((2.0 * i / n - 1.0) * math.atanh(s1)) / s1)
    xi[0], xi[-1] = 0.0, L
    return xi


def centres(faces):
    return 0.5 * (faces[1:] + faces[:-1])


# --------------------------------------------------------------- fields ----

def tgv_fields(n=64, u0=0.01):
    """Taylor-Green vortex at cell centres i + 1/2, k = 2 pi / n, rho from the
    pressure field p = -(u0^2/4)(cos 2kx + cos 2ky), p = cs^2 (rho - 1)."""
    k = 2 * math.pi / n
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x)  # [y][x]
    ux = -u0 * np.cos(k * X) * np.sin(k * Y)
    uy = u0 * np.sin(k * X) * np.cos(k * Y)
    rho = 1.0 - (u0 * u0 / 4.0) / CS2 * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    return rho, ux, uy


def poiseuille_profile(y, L, umax):
    return 4.0 * umax * y * (L - y) / (L * L)


def channel_fields(nx, yf, umax, noise=1e-3, seed_index=1):
    """Poiseuille parabola at the cell centres plus uniform +-noise on both
    velocity components, rho = 1."""
    L = yf[-1] - yf[0]
    yc = centres(yf)
    ny = len(yc)
    r = rng(seed_index)
    ux = np.repeat(poiseuille_profile(yc, L, umax)[:, None], nx, axis=1)
    ux = ux + r.uniform(-noise, noise, size=(ny, nx))
    uy = r.uniform(-noise, noise, size=(ny, nx))
    return np.ones((ny, nx)), ux, uy


def rb_fields(nx, yf, dT, T0, beta_g, noise=1e-3, seed_index=2):
    """Rayleigh-Benard initial state (sec. 5): fluid at rest, conductive profile
    T_c(y) = T0 + dT (1/2 - y/H) (hot bottom), hydrostatic density of the
    Boussinesq acceleration a_y = beta g (T - T0):  cs^2 d rho/dy = rho a_y,
    rho = 1 at mid height, i.e. rho = exp(-beta g dT (y - H/2)^2 / (2 H cs^2)),
    plus seeded uniform +-noise*dT on T."""
    H = yf[-1] - yf[0]
    yc = centres(yf) - yf[0]
    ny = len(yc)
    Tc = T0 + dT * (0.5 - yc / H)
    rho = np.exp(-beta_g * dT * (yc - 0.5 * H) ** 2 / (2.0 * H * CS2))
    r = rng(seed_index)
    T = np.repeat(Tc[:, None], nx, axis=1) + r.uniform(-noise * dT, noise * dT, size=(ny, nx))
    return np.repeat(rho[:, None], nx, axis=1), np.zeros((ny, nx)), np.zeros((ny, nx)), T


def rb3d_fields(nx, ny, zf, dT, T0, beta_g, noise=1e-3, seed_index=8):
    """The 3D Rayleigh-Benard initial state (z vertical): conductive T(z),
    hydrostatic density, seeded uniform +-noise*dT on T; arrays [nz][ny][nx]."""
    H = zf[-1] - zf[0]
    zc = centres(zf) - zf[0]
    nz = len(zc)
    Tc = T0 + dT * (0.5 - zc / H)
    rho = np.exp(-beta_g * dT * (zc - 0.5 * H) ** 2 / (2.0 * H * CS2))
    r = rng(seed_index)
    shape = (nz, ny, nx)
    T = np.broadcast_to(Tc[:, None, None], shape) + r.uniform(-noise * dT, noise * dT, size=shape)
    return (np.ascontiguousarray(np.broadcast_to(rho[:, None, None], shape)), np.zeros(shape), np.zeros(shape),
            np.zeros(shape), np.ascontiguousarray(T))


def rb3d_config(n, Ra, stretch, Pr=1.0, seed_index=8, cfl=1.0):
    """Cubic 3D Rayleigh-Benard cell (aspect 1, periodic sides, tanh-refined
    z), the recipe of sec. 5 as in rb_params."""
    P = rb_params(Ra, Pr, n, n, aspect=1.0, stretch=stretch, cfl=cfl)
    zf = P["yf"]
    rho, ux, uy, uz, T = rb3d_fields(n, n, zf, P["dT"], P["T0"], P["beta_g"], seed_index=seed_index)
    P.update(name=f"rb3d_{n}", nz=n, zf=zf, xf=P["xf"], yf=faces_uniform(n, P["L"]), rho=rho, ux=ux, uy=uy, uz=uz,
             T=T)
    return P


# ----------------------------------------------------------- parameters ----

def rb_params(Ra, Pr, nx, ny, aspect=1.0, stretch=2.0, U_ff=0.1, dT=1.0, tau_min=0.5, cfl=1.0):
    """Lattice parameters of a Rayleigh-Benard run.  The smaller of the two
    relaxation times is tau_min (the paper runs tau = tau_g = 1/2), the
    free-fall velocity sqrt(beta g dT H) is U_ff (about 0.1, sec. 5), so
    H = sqrt(Ra nu kappa) / U_ff.  dt = cfl * (smallest cell size)."""
    if Pr >= 1.0:
        kappa = tau_min * CS2
        nu = Pr * kappa
    else:
        nu = tau_min * CS2
        kappa = nu / Pr
    H = math.sqrt(Ra * nu * kappa) / U_ff
    L = aspect * H
    beta_g = U_ff * U_ff / (dT * H)
    yf = faces_tanh(ny, H, stretch)
    xf = faces_uniform(nx, L)
    dmin = min(float(np.min(np.diff(yf))), L / nx)
    return dict(nx=nx, ny=ny, tau=nu / CS2, tau_g=kappa / CS2, dt=cfl * dmin, beta_g=beta_g,
                T0=0.0, T_bottom=0.5 * dT, T_top=-0.5 * dT, H=H, L=L, xf=xf, yf=yf,
                Ra=Ra, Pr=Pr, nu=nu, kappa=kappa, dT=dT)


def tgv_config():
    """tgv64: lattice relaxation time 0.8 at dt = dx = 1, i.e. nu = 0.1 and the
    paper's tau = nu / cs^2 = 0.3."""
    n = 64
    nu = (0.8 - 0.5) * CS2
    rho, ux, uy = tgv_fields(n, 0.01)
    # FV time step 0.8: the linear stability limit of the semi-implicit + Heun
    # scheme for two-dimensional modes at this tau is about 0.95 dx.
    return dict(name="tgv64", nx=n, ny=n, tau=nu / CS2, dt=0.8, nu=nu, u0=0.01,
                xf=faces_uniform(n, n), yf=faces_uniform(n, n), rho=rho, ux=ux, uy=uy, steps=1000)


def channel_config(uniform=False):
    """channel: 256 x 512, tanh(2.0) wall-normal grid (or uniform for ST),
    nu = 1/30 (lattice relaxation 0.6), Re_bulk = U_b L / nu = 1000,
    U_max = 1.5 U_b, a_x = 8 nu U_max / L^2 (the parabola is the steady state)."""
    nx, ny, L = 256, 512, 512.0
    nu = (0.6 - 0.5) * CS2
    ub = 1000.0 * nu / L
    umax = 1.5 * ub
    yf = faces_uniform(ny, L) if uniform else faces_tanh(ny, L, 2.0)
    xf = faces_uniform(nx, float(nx))
    dmin = min(1.0, float(np.min(np.diff(yf))))
    rho, ux, uy = channel_fields(nx, yf, umax)
    return dict(name="channel", nx=nx, ny=ny, tau=nu / CS2, nu=nu, umax=umax, ax=8 * nu * umax / (L * L),
                dt=dmin, xf=xf, yf=yf, rho=rho, ux=ux, uy=uy, steps=20000)


def rb_config(n, Ra, stretch, Pr=1.0, seed_index=2, cfl=1.0):
    P = rb_params(Ra, Pr, n, n, aspect=1.0, stretch=stretch, cfl=cfl)
    rho, ux, uy, T = rb_fields(n, P["yf"], P["dT"], P["T0"], P["beta_g"], seed_index=seed_index)
    P.update(name=f"rb{n}", rho=rho, ux=ux, uy=uy, T=T)
    return P


def rb1024_config():
    return rb_config(1024, 1e8, 2.0)


def rb4096_config():
    return rb_config(4096, 1e10, 2.5, seed_index=5)


def serving_trace(n_requests=300, rate=20.0, seed_index=4, side=(128, 1024), ra=(1e6, 1e9),
                  prandtl=(0.7, 1.0, 7.0), steps=(2000, 20000)):
    """Poisson arrivals (mean `rate` per second) of Rayleigh-Benard requests:
    side log-uniform in [128, 1024] (square cells count, aspect 1), Ra
    log-uniform, Pr uniform over the set, steps uniform integer."""
    r = rng(seed_index)
    gaps = r.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(n_requests):
        n = int(round(math.exp(r.uniform(math.log(side[0]), math.log(side[1])))))
        out.append(dict(id=k, arrival=float(t[k]), n=n,
                        Ra=float(10 ** r.uniform(math.log10(ra[0]), math.log10(ra[1]))),
                        Pr=float(prandtl[r.integers(len(prandtl))]),
                        steps=int(r.integers(steps[0], steps[1] + 1))))
    return out
