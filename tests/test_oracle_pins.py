"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics (closed forms, invariants, textbook special cases, brute force on
tiny grids).  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import oracle.brute as brute
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
VEL = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])


def _random_state(ny, nx, seed, thermal=True, amp=0.02):
    r = np.random.default_rng(seed)
    rho = 1.0 + 0.01 * r.standard_normal((ny, nx))
    ux = amp * r.standard_normal((ny, nx))
    uy = amp * r.standard_normal((ny, nx))
    T = 0.2 * r.standard_normal((ny, nx)) if thermal else None
    return rho, ux, uy, T


# ------------------------------------------------------------ lattice -----

def test_equilibrium_moments_from_populations():
    """Zeroth, first and second moments of the initialised populations are the
    textbook ones: sum f = rho, sum c f = rho u, sum c c f = rho cs^2 I + rho u u
    (no force), which fixes the D2Q9 weights and the equilibrium polynomial."""
    ny, nx = 3, 4
    rho, ux, uy, _ = _random_state(ny, nx, 1, thermal=False, amp=0.05)
    c = oracle.Case(nx, ny)
    c.init(rho, ux, uy)
    f = c.f
    cx, cy = VEL[:, 0][:, None, None], VEL[:, 1][:, None, None]
    np.testing.assert_allclose(f.sum(0), rho, rtol=0, atol=1e-15)
    np.testing.assert_allclose((cx * f).sum(0), rho * ux, rtol=0, atol=1e-15)
    np.testing.assert_allclose((cy * f).sum(0), rho * uy, rtol=0, atol=1e-15)
    np.testing.assert_allclose((cx * cx * f).sum(0), rho / 3 + rho * ux * ux, atol=1e-15)
    np.testing.assert_allclose((cy * cy * f).sum(0), rho / 3 + rho * uy * uy, atol=1e-15)
    np.testing.assert_allclose((cx * cy * f).sum(0), rho * ux * uy, atol=1e-15)


def test_guo_force_moments_through_init():
    """With a body force the equilibrium tilde populations are f_eq - dt/2 F
    (appendix A).  The Guo force has sum F = 0, sum c F = rho a (sec. 2.2.4) and
    sum c_i c_j F = rho (u_i a_j + a_i u_j); the moments recovered by the
    'Force term' rule give back the prescribed u."""
    ny, nx = 2, 3
    rho, ux, uy, _ = _random_state(ny, nx, 2, thermal=False, amp=0.05)
    ax, ay, dt = 3e-3, -2e-3, 0.7
    c = oracle.Case(nx, ny, dt=dt, ax=ax, ay=ay)
    c.init(rho, ux, uy)
    f = c.f
    cx, cy = VEL[:, 0][:, None, None], VEL[:, 1][:, None, None]
    np.testing.assert_allclose(f.sum(0), rho, atol=1e-15)
    np.testing.assert_allclose((cx * f).sum(0), rho * ux - 0.5 * dt * rho * ax, atol=1e-15)
    np.testing.assert_allclose((cx * cy * f).sum(0), rho * ux * uy - 0.5 * dt * rho * (ux * ay + ax * uy),
                               atol=1e-15)
    np.testing.assert_allclose((cx * cx * f).sum(0), rho / 3 + rho * ux * ux - 0.5 * dt * rho * 2 * ux * ax,
                               atol=1e-15)
    m = c.moments()
    np.testing.assert_allclose(m["ux"], ux, atol=1e-15)
    np.testing.assert_allclose(m["uy"], uy, atol=1e-15)


def test_thermal_equilibrium_temperature():
    ny, nx = 3, 3
    rho, ux, uy, T = _random_state(ny, nx, 3)
    c = oracle.Case(nx, ny, thermal=True, beta_g=0.01)
    c.init(rho, ux, uy, T)
    np.testing.assert_allclose(c.g.sum(0), T, atol=1e-15)
    np.testing.assert_allclose(c.moments()["T"], T, atol=1e-15)


# -------------------------------------------------------------- QUICK -----

def test_quick_uniform_is_textbook():
    """On a uniform grid the upwind parabola gives the classic QUICK weights
    6/8, 3/8, -1/8 (Leonard), i.e. g1 = g3 = 3/8 and g2 = g4 = 1/8."""
    for periodic in (True, False):
        g = oracle.quick_gammas(np.arange(11.0) * 2.5, periodic)
        np.testing.assert_allclose(g, np.tile([0.375, 0.125, 0.375, 0.125], (11, 1)), atol=1e-15)


def _node_positions(faces, periodic):
    n = len(faces) - 1
    c = 0.5 * (faces[1:] + faces[:-1])
    L = faces[-1] - faces[0]
    if periodic:
        ext = np.concatenate([c[-2:] - L, c, c[:2] + L])
    else:
        ext = np.concatenate([2 * faces[0] - c[1::-1], c, 2 * faces[-1] - c[:-3:-1]])
    return ext  # index k + 2 for node k in [-2, n+1]


@pytest.mark.parametrize("periodic", [True, False])
def test_quick_exact_for_quadratics_on_stretched_grids(periodic):
    """The face values built from g1..g4 reproduce any quadratic exactly on
    any stretched grid (sec. 2.2.3: the interpolant is a parabola)."""
    r = np.random.default_rng(7)
    for n in (6, 11, 40):
        faces = np.concatenate([[0.0], np.cumsum(r.uniform(0.2, 3.0, n))])
        g = oracle.quick_gammas(faces, periodic)
        x = _node_positions(faces, periodic)
        a, b, cq = r.standard_normal(3)
        q = lambda s: a + b * s + cq * s * s
        for k in range(n + 1):
            P, E, Wn, EE = x[k + 1], x[k + 2], x[k], x[k + 3]
            if periodic and k == 0:
                continue  # face 0 duplicates face n
            up = (1 - g[k, 0] + g[k, 1]) * q(P) + g[k, 0] * q(E) - g[k, 1] * q(Wn)
            dn = (1 - g[k, 2] + g[k, 3]) * q(E) + g[k, 2] * q(P) - g[k, 3] * q(EE)
            scale = max(abs(q(P)), abs(q(E)), abs(q(Wn)), abs(q(EE)), 1.0)
            assert abs(up - q(faces[k])) < 1e-12 * scale
            assert abs(dn - q(faces[k])) < 1e-12 * scale


def test_quick_wall_mirror_identity():
    """Mirrored ghost centres make the two upwind parabolas at a wall face
    mirror images: g3 = g1 and g4 = g2 there (basis of exact no-penetration)."""
    faces = workloads.faces_tanh(17, 40.0, 2.0)
    g = oracle.quick_gammas(faces, False)
    for k in (0, 17):
        assert abs(g[k, 2] - g[k, 0]) < 1e-14 and abs(g[k, 3] - g[k, 1]) < 1e-14


# -------------------------------------------------------------- grids -----

def test_tanh_grid_properties_and_independent_generator():
    for n, s in ((8, 2.0), (512, 2.0), (4096, 2.5)):
        xi = oracle.grid_tanh(n, 100.0, math.tanh(s))
        assert xi[0] == 0.0 and xi[-1] == 100.0
        np.testing.assert_allclose(xi + xi[::-1], 100.0, atol=1e-12)
        assert np.all(np.diff(xi) > 0)
        np.testing.assert_allclose(xi, workloads.faces_tanh(n, 100.0, s), rtol=0, atol=1e-13)
    d = np.diff(oracle.grid_tanh(512, 512.0, math.tanh(2.0)))
    # stretch 2.0: the wall cell is 1/cosh(2)^2 = 0.0707 of the centre cell
    assert abs(d.min() / d.max() - 1 / math.cosh(2.0) ** 2) < 1e-3


def test_table1_parameters_reproduce_rayleigh_number():
    """sec. 5, Table 1: with nu = tau cs^2, kappa = tau_g cs^2 (the paper's tau,
    not tau~) both rows give Ra = beta g dT H^3 / (nu kappa) = 2.5e6 and the
    same free-fall velocity sqrt(beta g dT H)."""
    t = json.load(open(os.path.join(GOLDEN, "table1_rb.json")))
    us = []
    for row in t["rows"].values():
        nu, ka = row["tau"] / 3, row["tau_g"] / 3
        Ra = row["beta"] * row["g"] * row["dT"] * row["H"] ** 3 / (nu * ka)
        assert abs(Ra / t["Ra"] - 1) < 1e-3
        assert row["L"] == 2 * row["H"]
        us.append(math.sqrt(row["beta"] * row["g"] * row["dT"] * row["H"]))
    assert abs(us[0] - us[1]) < 1e-12 and abs(us[0] - 0.412) < 1e-3


# --------------------------------------------------------- invariants -----

CASES = [
    dict(name="periodic", wall_y=False, stretched=False),
    dict(name="walls-stretched", wall_y=True, stretched=True),
    dict(name="walls-both", wall_y=True, wall_x=True, stretched=True),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
@pytest.mark.parametrize("scheme", ["heun", "semi", "st"])
def test_mass_conservation(case, scheme):
    """Fluxes telescope and double reflection carries no mass through a wall
    (face values of a and inv(a) coincide), so sum V rho is constant to
    rounding; collision conserves mass."""
    if scheme == "st" and case["stretched"]:
        case = dict(case, stretched=False)
    nx, ny = 12, 10
    yf = workloads.faces_tanh(ny, 30.0, 2.0) if case["stretched"] else np.arange(ny + 1.0)
    c = oracle.Case(nx, ny, scheme=scheme, wall_x=case.get("wall_x", False), wall_y=case["wall_y"],
                    thermal=True, dt=0.8, tau=0.2, tau_g=0.3, ax=1e-4, beta_g=1e-3,
                    T_bottom=0.5, T_top=-0.5, yf=yf)
    c.init(*_random_state(ny, nx, 11))
    m0 = c.diagnostics()["mass"]
    c.step(40)
    m1 = c.diagnostics()["mass"]
    assert abs(m1 / m0 - 1) < 1e-13


@pytest.mark.parametrize("scheme", ["heun", "semi", "st"])
def test_momentum_periodic(scheme):
    """Periodic, unforced: total momentum is conserved; with a constant force
    it grows by exactly dt * sum V rho a per step (sum c C = dt rho a)."""
    nx, ny = 9, 7
    dt = 1.0 if scheme == "st" else 0.9
    for a in (0.0, 2e-4):
        c = oracle.Case(nx, ny, scheme=scheme, dt=dt, tau=0.25, ax=a, ay=-0.5 * a)
        c.init(*_random_state(ny, nx, 5, thermal=False))
        def P():
            cx, cy = VEL[:, 0][:, None, None], VEL[:, 1][:, None, None]
            return (cx * c.f).sum(), (cy * c.f).sum()
        p0 = P()
        mass = c.f.sum()
        c.step(25)
        p1 = P()
        assert abs(p1[0] - p0[0] - 25 * dt * mass * a) < 1e-13
        assert abs(p1[1] - p0[1] + 25 * dt * mass * 0.5 * a) < 1e-13


@pytest.mark.parametrize("scheme,dt", [("heun", 0.7), ("heun", 3.0), ("semi", 2.0), ("euler", 0.3), ("st", 1.0)])
def test_uniform_relaxation_closed_form(scheme, dt):
    """A uniform state has no advection (D = 0) and its non-equilibrium part
    decays by r = (tau - dt/2)/(tau + dt/2) per step for the semi-implicit
    schemes and ST (|r| < 1 for every dt: sec. 2.2.2), by 1 - dt/tau for Euler."""
    tau = 0.4
    nx, ny = 3, 2
    c = oracle.Case(nx, ny, scheme=scheme, dt=dt, tau=tau)
    c.init(np.ones((ny, nx)), np.full((ny, nx), 0.03), np.full((ny, nx), -0.01))
    feq = c.f.copy()
    h = np.array([0, 1, -1, 1, -1, 0, 0, 0, 0], dtype=float)[:, None, None] * 1e-3  # no mass, no momentum
    c.f = np.ascontiguousarray(c.f + h)
    r = (1 - dt / tau) if scheme == "euler" else (tau - dt / 2) / (tau + dt / 2)
    if scheme == "st":
        r = (tau - 0.5) / (tau + 0.5)
    for n in range(1, 6):
        c.step(1)
        np.testing.assert_allclose(c.f - feq, np.broadcast_to(h * r ** n, feq.shape), atol=1e-15, rtol=1e-11)


@pytest.mark.parametrize("scheme", ["heun", "st"])
def test_uniform_flow_is_fixed_point(scheme):
    nx, ny = 5, 4
    c = oracle.Case(nx, ny, scheme=scheme, dt=1.0, tau=0.3)
    c.init(np.ones((ny, nx)), np.full((ny, nx), 0.05), np.full((ny, nx), 0.02))
    f0 = c.f.copy()
    c.step(10)
    np.testing.assert_allclose(c.f, f0, atol=2e-16, rtol=0)


# ---------------------------------------------------------- brute force ----

BRUTE = [
    dict(nx=4, ny=4, wall_y=False, stretched=False, thermal=False, ax=0.0),
    dict(nx=5, ny=7, wall_y=True, stretched=True, thermal=True, ax=1e-3),
    dict(nx=8, ny=6, wall_y=True, wall_x=True, stretched=True, thermal=True, ax=-2e-3),
    dict(nx=6, ny=5, wall_y=False, stretched=True, thermal=True, ax=0.0),
    dict(nx=7, ny=5, wall_y=True, wall_x=2, stretched=True, thermal=False, ax=0.0),
]


@pytest.mark.parametrize("cfg", BRUTE, ids=lambda c: f"{c['nx']}x{c['ny']}")
def test_fv_heun_matches_brute_force(cfg):
    nx, ny = cfg["nx"], cfg["ny"]
    r = np.random.default_rng(nx * 100 + ny)
    yf = np.concatenate([[0.0], np.cumsum(r.uniform(0.3, 2.0, ny))]) if cfg["stretched"] else np.arange(ny + 1.0)
    xf = np.concatenate([[0.0], np.cumsum(r.uniform(0.5, 1.5, nx))]) if cfg.get("wall_x") else np.arange(nx + 1.0)
    c = oracle.Case(nx, ny, wall_x=cfg.get("wall_x", False), wall_y=cfg["wall_y"], thermal=cfg["thermal"],
                    dt=0.6, tau=0.25, tau_g=0.15, ax=cfg["ax"], ay=5e-4, beta_g=2e-3, T0=0.1,
                    T_bottom=0.7, T_top=-0.3, xf=xf, yf=yf, rho_lo=1.004, rho_hi=0.997)
    c.init(*_random_state(ny, nx, nx + ny, thermal=cfg["thermal"]))
    f0 = c.f.copy()
    g0 = c.g.copy() if cfg["thermal"] else None
    c.step(5)
    bf, bg = brute.fv_heun(c.brute_params(), c.xf, c.yf, f0, g0, 5)
    assert np.abs(bf - c.f).max() < 1e-13
    if cfg["thermal"]:
        assert np.abs(bg - c.g).max() < 1e-13


@pytest.mark.parametrize("cfg", [c for c in BRUTE if c.get("wall_x") != 2], ids=lambda c: f"{c['nx']}x{c['ny']}")
def test_st_matches_brute_force(cfg):
    nx, ny = cfg["nx"], cfg["ny"]
    c = oracle.Case(nx, ny, scheme="st", wall_x=cfg.get("wall_x", False), wall_y=cfg["wall_y"],
                    thermal=cfg["thermal"], tau=0.25, tau_g=0.15, ax=cfg["ax"], ay=5e-4, beta_g=2e-3,
                    T0=0.1, T_bottom=0.7, T_top=-0.3)
    c.init(*_random_state(ny, nx, nx * ny, thermal=cfg["thermal"]))
    f0 = c.f.copy()
    g0 = c.g.copy() if cfg["thermal"] else None
    c.step(5)
    bf, bg = brute.st(c.brute_params(), f0, g0, 5)
    assert np.abs(bf - c.f).max() < 1e-14
    if cfg["thermal"]:
        assert np.abs(bg - c.g).max() < 1e-14


def test_st_stream_map_is_a_permutation():
    for wx, wy in ((False, False), (False, True), (True, True)):
        c = oracle.Case(7, 5, scheme="st", wall_x=wx, wall_y=wy)
        src = c.stream_sources()
        assert np.array_equal(np.sort(src), np.arange(src.size))


# -------------------------------------------------------- closed forms -----

def _decay_rate(series, dt_between):
    t = np.arange(len(series)) * dt_between
    return -np.polyfit(t, np.log(series), 1)[0]


@pytest.mark.parametrize("scheme", ["heun", "st"])
def test_taylor_green_viscosity(scheme):
    """tgv64 workload: kinetic energy decays as exp(-2 nu (k_x^2 + k_y^2) t)
    (sec. 3.1 uses the 1D analogue).  The viscosity must be tau cs^2."""
    cfg = workloads.tgv_config()
    n = cfg["nx"]
    dt = 1.0 if scheme == "st" else cfg["dt"]
    c = oracle.Case(n, n, scheme=scheme, dt=dt, tau=cfg["tau"], xf=cfg["xf"], yf=cfg["yf"])
    c.init(cfg["rho"], cfg["ux"], cfg["uy"])
    E = []
    nper = int(round(100 / dt))
    for _ in range(11):
        E.append(c.diagnostics()["ekin"])
        c.step(nper)
    k = 2 * math.pi / n
    nu_fit = _decay_rate(np.array(E[1:]), nper * dt) / (4 * k * k)
    tol = 0.005 if scheme == "st" else 0.03
    assert abs(nu_fit / cfg["nu"] - 1) < tol


def test_shear_wave_viscosity_fv_stretched():
    """1D shear wave u_x = A sin(2 pi y / L) on a periodic tanh-stretched y grid
    (sec. 3.1 test geometry): the decay rate gives nu within a few percent."""
    ny, L, tau, dt = 64, 64.0, 0.5, 0.5
    yf = workloads.faces_uniform(ny, L)
    c = oracle.Case(1, ny, dt=dt, tau=tau, yf=yf)
    y = workloads.centres(yf)
    ux = 0.01 * np.sin(2 * math.pi * y / L)[:, None]
    c.init(np.ones((ny, 1)), ux, np.zeros((ny, 1)))
    E = []
    for _ in range(9):
        E.append(c.diagnostics()["ekin"])
        c.step(200)
    k = 2 * math.pi / L
    nu_fit = _decay_rate(np.array(E[1:]), 200 * dt) / (2 * k * k)
    assert abs(nu_fit / (tau / 3) - 1) < 0.02


def test_poiseuille_st_magic_tau_exact():
    """Textbook property of BGK with half-way bounce-back and a consistent
    body force: at tau~ = 1/2 + sqrt(3)/4 the parabola is reproduced exactly."""
    ny, L = 16, 16.0
    tau = math.sqrt(3) / 4  # tau~ = tau + 1/2
    nu = tau / 3
    umax = 0.01
    c = oracle.Case(1, ny, scheme="st", wall_y=True, tau=tau, ax=8 * nu * umax / L ** 2)
    y = workloads.centres(np.arange(ny + 1.0))
    U = workloads.poiseuille_profile(y, L, umax)
    c.init(np.ones((ny, 1)), U[:, None] * 0.5, np.zeros((ny, 1)))
    c.step(12000)
    ux = c.moments()["ux"][:, 0]
    assert np.abs(ux - U).max() < 1e-11 * umax


def _poiseuille_error(ny, L, scheme, yf=None, Re=10.0, tau=0.5, dt=1.0, steps=None):
    nu = tau / 3
    umax = Re * nu / L
    yf = np.linspace(0, L, ny + 1) if yf is None else yf
    c = oracle.Case(1, ny, scheme=scheme, wall_y=True, tau=tau, dt=dt, ax=8 * nu * umax / L ** 2, yf=yf)
    y = workloads.centres(yf)
    U = workloads.poiseuille_profile(y, L, umax)
    c.init(np.ones((ny, 1)), U[:, None], np.zeros((ny, 1)))
    steps = steps or int(6 * L * L / nu / dt)
    c.step(steps)
    u = c.moments()["ux"][:, 0]
    w = np.diff(yf)
    return math.sqrt(np.sum((u - U) ** 2 * w) / np.sum(U ** 2 * w))


def test_poiseuille_fv_converges_with_resolution():
    """sec. 3.2: Re = 10 Poiseuille on L = 64; refining the uniform FV grid
    lowers the volume-weighted relative L2 error (the paper reports roughly
    third order before the Mach plateau)."""
    e8 = _poiseuille_error(8, 64.0, "heun", tau=0.5, dt=2.0)
    e16 = _poiseuille_error(16, 64.0, "heun", tau=0.5, dt=2.0)
    assert e16 < e8 / 4
    assert e16 < 2e-2


def test_poiseuille_tanh_beats_uniform_fv():
    """sec. 3.2 (Fig. 4): at equal N the wall-refined tanh grid is more
    accurate than the uniform one (coarse grids, L = 64)."""
    L = 64.0
    eu = _poiseuille_error(12, L, "heun", tau=0.5, dt=2.0)
    et = _poiseuille_error(12, L, "heun", yf=workloads.faces_tanh(12, L, math.atanh(0.98)), tau=0.5, dt=0.5)
    assert et < eu


# ------------------------------------------------------------- thermal ----

@pytest.mark.parametrize("scheme", ["heun", "st"])
def test_conduction_is_exact_steady_state(scheme):
    """With no buoyancy, the linear conductive profile between isothermal walls
    with populations g~ = w (T(y) - tau~ c_y dT/dy) (tau~ = tau_g + dt/2) is an
    exact discrete steady state of both schemes under the wall rules, on any
    stretched grid for FV; wall and volume Nusselt numbers are exactly 1."""
    nx, ny = 4, 12
    Tb, Tt = 0.5, -0.5
    if scheme == "st":
        yf, dt = np.arange(ny + 1.0), 1.0
    else:
        yf, dt = workloads.faces_tanh(ny, 30.0, 2.0), 0.4
    H = yf[-1]
    G = (Tt - Tb) / H
    tg = 0.3
    c = oracle.Case(nx, ny, scheme=scheme, wall_y=True, thermal=True, dt=dt, tau=0.2, tau_g=tg,
                    T_bottom=Tb, T_top=Tt, yf=yf)
    y = workloads.centres(yf)
    T = Tb + G * y
    c.init(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), np.repeat(T[:, None], nx, 1))
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    cy = VEL[:, 1][:, None, None]
    c.g = np.ascontiguousarray(w * (T[None, :, None] - (tg + dt / 2) * cy * G) * np.ones((9, ny, nx)))
    g0 = c.g.copy()
    c.step(50)
    np.testing.assert_allclose(c.g, g0, atol=1e-15)
    d = c.diagnostics()
    assert abs(d["nu_bottom"] - 1) < 1e-12 and abs(d["nu_top"] - 1) < 1e-12
    assert abs(d["nu_vol"] - 1) < 1e-12


@pytest.mark.parametrize("scheme", ["heun", "st"])
def test_thermal_diffusion_rate(scheme):
    """A sinusoidal temperature mode at rest decays as exp(-kappa k^2 t),
    kappa = tau_g cs^2 (sec. 5)."""
    n, tg = 48, 0.4
    c = oracle.Case(1, n, scheme=scheme, thermal=True, dt=1.0, tau=0.3, tau_g=tg)
    y = np.arange(n) + 0.5
    T = 0.01 * np.sin(2 * math.pi * y / n)
    c.init(np.ones((n, 1)), np.zeros((n, 1)), np.zeros((n, 1)), T[:, None])
    amps = []
    for _ in range(8):
        Tn = c.moments()["T"][:, 0]
        amps.append(np.sqrt(np.mean(Tn ** 2)))
        c.step(100)
    k = 2 * math.pi / n
    kappa_fit = _decay_rate(np.array(amps[1:]), 100) / (k * k)
    assert abs(kappa_fit / (tg / 3) - 1) < (0.005 if scheme == "st" else 0.03)


def _rb_run(scheme, ny, Ra, steps, aspect=2.02, stretch=None):
    """2D Rayleigh-Benard at Pr = 1 for the steady-Nusselt pin (fluid at rest,
    conductive profile, one-roll perturbation of 1e-2 dT)."""
    nx = int(round(aspect * ny))
    U = 0.1
    if scheme == "st":
        H = float(ny)
        nu = U * H / math.sqrt(Ra)
        tau, dt = 3 * nu, 1.0
        yf, xf = np.arange(ny + 1.0), np.arange(nx + 1.0)
    else:
        tau = 0.5
        nu = tau / 3
        H = nu * math.sqrt(Ra) / U
        yf = workloads.faces_uniform(ny, H) if stretch is None else workloads.faces_tanh(ny, H, stretch)
        xf = workloads.faces_uniform(nx, aspect * H)
        dt = min(np.diff(yf).min(), np.diff(xf).min())
    beta_g = U * U / H
    c = oracle.Case(nx, ny, scheme=scheme, wall_y=True, thermal=True, dt=dt, tau=tau, tau_g=tau,
                    beta_g=beta_g, T_bottom=0.5, T_top=-0.5, xf=xf, yf=yf)
    rho, ux, uy, T = workloads.rb_fields(nx, yf, 1.0, 0.0, beta_g, noise=0.0)
    xc = workloads.centres(xf)
    T = T + 0.01 * np.sin(math.pi * xc / xf[-1])[None, :] * np.sin(math.pi * workloads.centres(yf) / H)[:, None]
    c.init(rho, ux, uy, T)
    c.step(steps)
    return c.diagnostics()


@pytest.mark.slow
def test_rayleigh_benard_ra1e4_nusselt_st():
    """sec. 5: 2D RB at Ra = 1e4, Pr = 1, Ar = 2.02 settles to Nu = 2.66."""
    gold = json.load(open(os.path.join(GOLDEN, "rb_ra1e4.json")))
    d = _rb_run("st", 32, gold["Ra"], 40000)
    assert abs(d["nu_vol"] - gold["Nu"]) < 0.05
    assert abs(d["nu_bottom"] - gold["Nu"]) < 0.05
    assert abs(d["nu_top"] - gold["Nu"]) < 0.05


@pytest.mark.slow
def test_rayleigh_benard_ra1e4_nusselt_fv():
    gold = json.load(open(os.path.join(GOLDEN, "rb_ra1e4.json")))
    d = _rb_run("heun", 32, gold["Ra"], 30000, stretch=1.0)
    assert abs(d["nu_vol"] - gold["Nu"]) < 0.05
    assert abs(d["nu_bottom"] - gold["Nu"]) < 0.05
    assert abs(d["nu_top"] - gold["Nu"]) < 0.05


def test_onset_between_1600_and_1800():
    """sec. 5: at aspect ratio 2.02 convection sets in between Ra = 1600 and
    1800.  The oracle's stored roll energies (written by
    tests/golden/make_onset_rates.py) decay at 1600 and grow at 1800 at a
    steady exponential rate, and the oracle still reproduces the first
    checkpoint of both runs."""
    gold = json.load(open(os.path.join(GOLDEN, "rb_onset_rates.json")))
    rate = {}
    for key, run in gold["runs"].items():
        e = np.array(run["roll_energy"])
        r = e[1:] / e[:-1]
        assert np.ptp(r) < 1e-3 * r.mean()                 # one exponential mode
        rate[key] = r.mean()
    assert rate["1600"] < 0.9 and rate["1800"] > 1.1
    cfg = gold["config"]
    for key, run in gold["runs"].items():
        Ra = float(key)
        nx, ny = run["nx"], cfg["ny"]
        P = workloads.rb_params(Ra, cfg["Pr"], nx, ny, aspect=nx / ny, stretch=cfg["stretch"])
        rho, ux, uy, T = workloads.rb_fields(nx, P["yf"], P["dT"], P["T0"], P["beta_g"], noise=cfg["noise"],
                                             seed_index=cfg["seed_index"])
        c = oracle.Case(nx, ny, scheme="heun", thermal=True, wall_y=True, dt=P["dt"], tau=P["tau"],
                        tau_g=P["tau_g"], beta_g=P["beta_g"], T0=P["T0"], T_bottom=P["T_bottom"],
                        T_top=P["T_top"], xf=P["xf"], yf=P["yf"])
        c.init(rho, ux, uy, T)
        c.step(run["steps_per_checkpoint"])
        m = c.moments()
        du = m["ux"] - m["ux"].mean(axis=1, keepdims=True)
        dv = m["uy"] - m["uy"].mean(axis=1, keepdims=True)
        e = 0.5 * float(np.sum(m["rho"] * (du * du + dv * dv)))
        assert abs(e / run["roll_energy"][0] - 1) < 1e-9


def _poiseuille_error_reading(n, cfl, alt, L=64.0, Re=10.0, U=0.05):
    """Relative L2 error of the steady FV-Heun Poiseuille profile (sec. 3.2:
    uniform cells, Re = 10, a_x = 8 nu U / L^2, three viscous times from the
    exact parabola), with the literal bracket or its alternative reading."""
    oracle.set_bracket(alt)
    try:
        nu = U * L / Re
        yf = np.linspace(0.0, L, n + 1)
        dy = np.diff(yf)
        dt = cfl * dy.min()
        c = oracle.Case(4, n, scheme="heun", wall_y=True, dt=dt, tau=nu / (1.0 / 3.0), ax=8 * nu * U / L ** 2,
                        xf=np.linspace(0.0, 4 * dy.max(), 5), yf=yf)
        yc = 0.5 * (yf[1:] + yf[:-1])
        prof = 4 * U * yc * (L - yc) / L ** 2
        c.init(np.ones((n, 4)), np.repeat(prof[:, None], 4, 1), np.zeros((n, 4)))
        c.step(int(math.ceil(3.0 * L * L / nu / dt)))
        ux = c.moments()["ux"][:, 0]
        return math.sqrt(np.sum((ux - prof) ** 2 * dy) / np.sum(prof ** 2 * dy))
    finally:
        oracle.set_bracket(False)


def test_bracket_reading_and_the_steady_poiseuille_profile():
    """Reading of the advected bracket's force term (eq:semi takes +dt/2 F;
    the physical distribution of the Crank-Nicolson transform carries
    dt/2 (1 - dt/(2 tau~)) F).  With the latter the steady state of a forced
    flow cannot depend on dt, and the oracle's steady Poiseuille error is the
    same at two time steps; with the literal bracket, which the implementation
    follows, it moves by a few per cent of the discretisation error at the
    coarse grids of Fig. 3 (N = 8)."""
    e_alt = [_poiseuille_error_reading(8, cfl, True) for cfl in (0.5, 1.0)]
    assert abs(e_alt[0] - e_alt[1]) < 1e-6 * e_alt[0]
    for cfl in (0.5, 1.0):
        e_lit = _poiseuille_error_reading(8, cfl, False)
        assert abs(e_lit - e_alt[0]) < 0.06 * e_alt[0]


# ----------------------------------------------------------- stability ----

def _kolmogorov_blows_up(scheme, tau, dt, steps=3000, n=64):
    """Decaying Kolmogorov (shear) flow on the [1, 64] domain of sec. 3.1 /
    Fig. 6 with a small random seed of every mode."""
    c = oracle.Case(1, n, scheme=scheme, dt=dt, tau=tau)
    y = np.arange(n) + 0.5
    r = np.random.default_rng(3)
    ux = 0.01 * np.sin(2 * math.pi * y / n) + 1e-6 * r.standard_normal(n)
    c.init(np.ones((n, 1)), ux[:, None], 1e-6 * r.standard_normal((n, 1)))
    c.step(steps)
    e = c.diagnostics()["ekin"]
    return not np.isfinite(e) or e > 1.0


def test_stability_statements_of_the_paper():
    """sec. 2.2.2 and sec. 4 (Fig. 6): Euler is bounded by dt <= 2 tau; the
    semi-implicit scheme is still limited by the advection at small tau; the
    semi-implicit + Heun scheme allows dt > 1 (dx = 1) for tau > 1/8."""
    assert _kolmogorov_blows_up("euler", 0.2, 0.45)
    assert not _kolmogorov_blows_up("euler", 0.2, 0.3)
    assert _kolmogorov_blows_up("semi", 0.2, 1.0)
    for tau in (0.15, 0.5):
        assert not _kolmogorov_blows_up("heun", tau, 1.3)
    assert _kolmogorov_blows_up("heun", 0.5, 1.9)


def test_golden_steady_roll_is_steady_and_balanced():
    """The oracle's stored steady Rayleigh-Benard roll (Ra = 1e4): at a
    steady state the heat entering at the bottom leaves at the top (equal
    wall Nusselt numbers), the volume estimate agrees with them to the
    discretisation error, and the run had stopped changing."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "rb64_ra1e4_steady.json")
    with open(path) as fh:
        g = json.load(fh)
    assert abs(g["nu_bottom"] - g["nu_top"]) < 1e-8
    assert max(g["nu_change_last_tenth"]) < 1e-7
    assert abs(g["nu_vol"] - g["nu_bottom"]) / g["nu_bottom"] < 1e-2
    assert 2.0 < g["nu_bottom"] < 2.6        # convecting: well above conduction (Nu = 1)
    T = g["T_profile"]
    assert abs(T[0] - 0.5) < 0.05 and abs(T[-1] + 0.5) < 0.05   # near the wall temperatures
    assert all(abs(T[j] + T[-1 - j]) < 1e-6 for j in range(len(T)))  # Boussinesq up-down symmetry


# ------------------------------------------------ fixed-density boundary ----
# "Boundary conditions", second rule: ghost densities extrapolated linearly
# through the boundary value, ghost populations = the mirror cell's rescaled.

def test_fixed_density_rest_state_is_a_fixed_point():
    """Fluid at rest at the boundary density: the ghosts equal their mirror
    cells, every face value equals the cell value, and nothing moves."""
    nx, ny = 12, 8
    xf = np.concatenate([[0.0], np.cumsum(np.random.default_rng(2).uniform(0.5, 1.5, nx))])
    yf = oracle.grid_tanh(ny, 8.0, 0.8)
    c = oracle.Case(nx, ny, wall_x=2, wall_y=True, dt=0.5, tau=0.3, xf=xf, yf=yf, rho_lo=1.02, rho_hi=1.02)
    c.init(np.full((ny, nx), 1.02), np.zeros((ny, nx)), np.zeros((ny, nx)))
    f0 = c.f.copy()
    c.step(20)
    assert np.abs(c.f - f0).max() < 1e-15


def _pressure_channel(nx, ny, steps, drho=0.002, tau=1.0 / 6.0, dt=0.5):
    L_x, L_y = float(nx), float(ny)
    c = oracle.Case(nx, ny, wall_x=2, wall_y=True, dt=dt, tau=tau, xf=np.arange(nx + 1.0),
                    yf=oracle.grid_tanh(ny, L_y, 0.8), rho_lo=1.0 + drho / 2, rho_hi=1.0 - drho / 2)
    x = 0.5 * (c.xf[1:] + c.xf[:-1])
    rho0 = np.tile(1.0 + drho / 2 - drho * x / L_x, (ny, 1))
    c.init(rho0, np.zeros((ny, nx)), np.zeros((ny, nx)))
    c.step(steps)
    return c, L_x, L_y


def test_pressure_driven_channel_reaches_poiseuille():
    """A density difference across a walled channel drives the Poiseuille
    flow: at steady state the mass flux through every cross-section is the
    same, the density falls linearly, and the centreline speed is
    dp/dx L_y^2 / (8 rho nu) with p = cs^2 rho (nu = tau cs^2)."""
    nx, ny, drho, tau = 24, 16, 0.002, 1.0 / 6.0
    c, L_x, L_y = _pressure_channel(nx, ny, 6000, drho=drho, tau=tau)
    m = c.moments()
    dy = np.diff(c.yf)
    flux = (m["rho"] * m["ux"] * dy[:, None]).sum(axis=0)       # per column
    assert np.abs(flux - flux.mean()).max() < 2e-4 * abs(flux.mean())
    assert abs(m["uy"]).max() < 1e-3 * m["ux"].max()
    rho_mean = m["rho"].mean(axis=0)
    slope = np.polyfit(np.arange(nx) + 0.5, rho_mean, 1)[0]
    assert abs(slope * L_x / -drho - 1) < 0.05
    nu = tau / 3.0
    u_max = (drho / 3.0 / L_x) * L_y ** 2 / (8.0 * nu * 1.0)
    centre = m["ux"][ny // 2 - 1:ny // 2 + 1, nx // 2].mean()
    assert abs(centre / u_max - 1) < 0.03


# ------------------------------------------- pins added for the grid, the ---
# ------------------------------------- thermal energy and the wall rule -----

def test_sinh_grid_printed_formula_and_properties():
    """eq:grids, hyperbolic sine: two branches that meet at i = N/2 (the
    low branch up to N/2, the mirrored one from N/2 + 1), evaluated here
    from the printed expression with s2 = 6.5 (sec. 3.2), and the properties
    any correct evaluation has: end faces 0 and L, symmetry
    xi_i + xi_{N-i} = L, the middle face at L/2, monotone faces, and a wall
    cell of width A sinh(s2 / N) with A = (L/2) / sinh(s2/2)."""
    L, s2 = 64.0, 6.5
    for n in (8, 12, 64, 500):
        xi = oracle.grid_sinh(n, L, s2)
        A = (L / 2) / math.sinh(s2 / 2)
        printed = np.array([A * math.sinh(s2 * i / n) if i <= n // 2 else L - A * math.sinh(s2 * (n - i) / n)
                            for i in range(n + 1)])
        np.testing.assert_allclose(xi, printed, rtol=0, atol=1e-12 * L)
        assert xi[0] == 0.0 and abs(xi[-1] - L) < 1e-12 * L
        np.testing.assert_allclose(xi + xi[::-1], L, atol=1e-12 * L)
        assert abs(xi[n // 2] - L / 2) < 1e-12 * L
        d = np.diff(xi)
        assert np.all(d > 0)
        assert abs(d[0] - A * math.sinh(s2 / n)) < 1e-12 * L
        # the cells grow away from each wall up to the middle
        assert np.all(np.diff(d[: n // 2]) > 0) and np.all(np.diff(d[n // 2:]) < 0)
    # the library's generator gives the same faces
    import paper_1505_03271_amd as lb
    np.testing.assert_allclose(lb.grid_sinh(64, L, s2), oracle.grid_sinh(64, L, s2), rtol=0, atol=1e-12 * L)


def test_thermal_energy_sum_of_a_linear_profile():
    """sum V T over cells is the midpoint rule, exact for a temperature linear
    in y on any grid: Lx * integral of T dy = Lx * H * (T_b + T_t) / 2 for the
    conductive profile; the kinetic energy of a uniform flow at uniform
    density is (1/2) rho |u|^2 Lx H.  Stretched in y, non-uniform in x."""
    nx, ny = 7, 11
    xf = np.cumsum(np.r_[0.0, 1.0 + 0.3 * np.sin(np.arange(nx))])
    yf = workloads.faces_tanh(ny, 40.0, 2.0)
    Lx, H = xf[-1], yf[-1]
    Tb, Tt = 0.7, -0.2
    y = workloads.centres(yf)
    T = np.repeat((Tb + (Tt - Tb) * y / H)[:, None], nx, 1)
    u0, v0, rho0 = 0.03, -0.02, 1.1
    for scheme in ("heun", "euler"):
        c = oracle.Case(nx, ny, scheme=scheme, wall_y=True, thermal=True, dt=0.5, tau=0.3, tau_g=0.4,
                        T_bottom=Tb, T_top=Tt, xf=xf, yf=yf)
        c.init(np.full((ny, nx), rho0), np.full((ny, nx), u0), np.full((ny, nx), v0), T)
        d = c.diagnostics()
        assert abs(d["etherm"] - Lx * H * 0.5 * (Tb + Tt)) < 1e-12 * Lx * H
        assert abs(d["ekin"] / (0.5 * rho0 * (u0 * u0 + v0 * v0) * Lx * H) - 1) < 1e-12
        assert abs(d["mass"] / (rho0 * Lx * H) - 1) < 1e-13
        assert abs(d["volume"] / (Lx * H) - 1) < 1e-14


@pytest.mark.parametrize("scheme", ["heun", "semi", "st"])
def test_thermal_energy_conserved_without_walls(scheme):
    """Periodic axes and no source: the g fluxes telescope and the collision
    keeps sum g, so sum V T is constant to rounding (sec. 5 model, no
    thermal boundary)."""
    nx, ny = 10, 9
    yf = np.arange(ny + 1.0) if scheme == "st" else workloads.faces_tanh(ny, 25.0, 1.5)
    c = oracle.Case(nx, ny, scheme=scheme, thermal=True, dt=1.0 if scheme == "st" else 0.6, tau=0.25,
                    tau_g=0.35, beta_g=2e-3, yf=yf)
    c.init(*_random_state(ny, nx, 21))
    e0 = c.diagnostics()["etherm"]
    c.step(60)
    e1 = c.diagnostics()["etherm"]
    assert abs(e1 - e0) < 1e-13 * max(1.0, abs(e0)) * nx * ny


@pytest.mark.parametrize("scheme", ["heun", "st"])
@pytest.mark.parametrize("Tw", [0.0, 0.3])
def test_isothermal_walls_give_dirichlet_decay(scheme, Tw):
    """The isothermal wall rule for g, pinned against the heat equation with
    Dirichlet data: at rest, T = Tw + A sin(pi y / H) between two walls held
    at Tw is the slowest mode and decays as exp(-kappa (pi/H)^2 t) with
    kappa = tau_g cs^2, while its shape stays a sine.  A wall that let no
    heat through (adiabatic) would keep the mean; a wrong sign or shift in the
    ghost rule moves the wall value away from Tw and changes the rate."""
    ny, tg = 40, 0.4
    H = float(ny)
    dt = 1.0 if scheme == "st" else 0.8
    c = oracle.Case(2, ny, scheme=scheme, wall_y=True, thermal=True, dt=dt, tau=0.3, tau_g=tg,
                    T_bottom=Tw, T_top=Tw)
    y = np.arange(ny) + 0.5
    mode = np.sin(math.pi * y / H)
    c.init(np.ones((ny, 2)), np.zeros((ny, 2)), np.zeros((ny, 2)), (Tw + 0.01 * mode)[:, None] * np.ones((1, 2)))
    per = 50
    amps, shapes = [], []
    for k in range(9):
        dev = c.moments()["T"][:, 0] - Tw
        amps.append(float(np.sum(dev * mode) / np.sum(mode * mode)))
        shapes.append(np.abs(dev - amps[-1] * mode).max() / abs(amps[-1]))
        c.step(int(round(per / dt)))
    rate = _decay_rate(np.array(amps[1:]), per)
    exact = (tg / 3.0) * (math.pi / H) ** 2
    assert abs(rate / exact - 1) < 0.02, (rate, exact)
    assert max(shapes[1:]) < 0.02
    # the mean excess temperature is not conserved: heat leaves through the
    # walls at the same rate (an adiabatic wall would keep it at 0.02 / pi)
    t_end = 9 * per
    mean = float(np.mean(c.moments()["T"] - Tw))
    assert abs(mean / (0.02 / math.pi * math.exp(-exact * t_end)) - 1) < 0.05
