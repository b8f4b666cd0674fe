"""Pins of the 3D (D3Q19) FV oracle: closed forms, invariants and an
independent brute-force recomputation (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute

# the oracle's population order (rest, axes, edges; opposite pairs adjacent)
ORDER = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
C = np.array(ORDER, dtype=float)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _fields(n, seed, amp=0.02, thermal=True):
    r = np.random.default_rng(seed)
    nx, ny, nz = n
    s = (nz, ny, nx)
    out = [1.0 + 0.01 * r.standard_normal(s)] + [amp * r.standard_normal(s) for _ in range(3)]
    out.append(0.3 * r.uniform(-1, 1, s) if thermal else None)
    return out


def test_d3q19_lattice_isotropy():
    assert abs(W.sum() - 1) < 1e-15
    assert np.abs(W @ C).max() < 1e-15
    np.testing.assert_allclose(np.einsum("a,ai,aj->ij", W, C, C), np.eye(3) / 3, atol=1e-15)
    m4 = np.einsum("a,ai,aj,ak,al->ijkl", W, C, C, C, C)
    d = np.eye(3)
    iso = (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)) / 9
    np.testing.assert_allclose(m4, iso, atol=1e-15)


def test_init_moments_and_momentum_flux():
    n = (5, 4, 3)
    rho, ux, uy, uz, T = _fields(n, 1)
    c = oracle.Case3D(*n, thermal=True, dt=0.5, tau=0.3)
    c.init(rho, ux, uy, uz, T)
    m = c.moments()
    for k, v in (("rho", rho), ("ux", ux), ("uy", uy), ("uz", uz), ("T", T)):
        np.testing.assert_allclose(m[k], v, rtol=0, atol=1e-14)
    # second moment of the equilibrium: rho cs^2 I + rho u u
    Pi = np.einsum("ai,aj,a...->ij...", C, C, c.f)
    u = np.stack([ux, uy, uz])
    expect = rho * (np.eye(3)[:, :, None, None, None] / 3 + u[:, None] * u[None, :])
    np.testing.assert_allclose(Pi, expect, atol=1e-14)


@pytest.mark.parametrize("walls", [(False, False, True), (True, True, True)])
def test_fv_heun_3d_matches_brute_force(walls):
    n = (3, 4, 5)
    r = np.random.default_rng(7)
    faces = [np.concatenate([[0.0], np.cumsum(r.uniform(0.5, 1.5, k))]) for k in n]
    c = oracle.Case3D(*n, walls=walls, thermal=True, dt=0.6, tau=0.25, tau_g=0.15, a=(1e-3, -5e-4, 2e-4),
                      beta_g=2e-3, T0=0.1, T_bottom=0.7, T_top=-0.3, xf=faces[0], yf=faces[1], zf=faces[2])
    c.init(*_fields(n, 9))
    f0, g0 = c.f.copy(), c.g.copy()
    c.step(2)
    bf, bg = brute.fv_heun_3d(c.brute_params(), faces, f0, g0, 2, ORDER)
    assert np.abs(bf - c.f).max() < 1e-13
    assert np.abs(bg - c.g).max() < 1e-13


def test_mass_conservation_and_fixed_point():
    n = (6, 5, 7)
    c = oracle.Case3D(*n, walls=(False, True, True), thermal=True, dt=0.5, tau=0.3, tau_g=0.2, beta_g=1e-3,
                      T_bottom=0.5, T_top=-0.5, zf=oracle.grid_tanh(7, 7.0, 0.8))
    c.init(*_fields(n, 3))
    m0 = c.diagnostics()["mass"]
    c.step(20)
    assert abs(c.diagnostics()["mass"] - m0) < 1e-13 * m0
    # uniform flow in a periodic box is a fixed point
    u = oracle.Case3D(4, 4, 4, dt=0.7, tau=0.2)
    s = (4, 4, 4)
    u.init(np.full(s, 1.01), np.full(s, 0.03), np.full(s, -0.02), np.full(s, 0.01))
    f0 = u.f.copy()
    u.step(10)
    assert np.abs(u.f - f0).max() < 1e-15


@pytest.mark.parametrize("dt", [0.4, 2.5])
def test_uniform_relaxation_closed_form(dt):
    """D = 0 for a uniform state: f~ - f_eq decays by (tau - dt/2)/(tau + dt/2) per step."""
    s = (4, 4, 4)
    tau = 0.3
    c = oracle.Case3D(4, 4, 4, dt=dt, tau=tau)
    c.init(np.ones(s), np.zeros(s), np.zeros(s), np.zeros(s))
    feq = c.f.copy()
    # a non-equilibrium part with no mass and no momentum: a traceless second moment
    dev = W[:, None, None, None] * (C[:, 0] * C[:, 1])[:, None, None, None] * np.ones((19,) + s) * 0.01
    c.f = feq + dev
    c.step(3)
    r = (tau - dt / 2) / (tau + dt / 2)
    np.testing.assert_allclose(c.f - feq, dev * r ** 3, atol=1e-16)


def test_shear_wave_viscosity_3d():
    """u_x(z) = A sin(2 pi z / L) decays as exp(-nu k^2 t) with nu = tau cs^2."""
    L, tau, dt = 32, 0.25, 0.5
    s = (L, 4, 4)
    z = (np.arange(L) + 0.5)[:, None, None] * np.ones(s)
    c = oracle.Case3D(4, 4, L, dt=dt, tau=tau)
    c.init(np.ones(s), 0.01 * np.sin(2 * math.pi * z / L), np.zeros(s), np.zeros(s))
    k = 2 * math.pi / L
    amps, ts = [], []
    for q in range(6):
        if q:
            c.step(100)
        ts.append(q * 100 * dt)
        ux = c.moments()["ux"][:, 0, 0]
        amps.append(np.dot(ux, np.sin(2 * math.pi * (np.arange(L) + 0.5) / L)) * 2 / L)
    nu = -np.polyfit(ts[1:], np.log(amps[1:]), 1)[0] / (k * k)
    assert abs(nu / (tau / 3) - 1) < 0.02


def test_conduction_is_exact_steady_state_3d():
    n = (4, 4, 12)
    H = 24.0
    zf = oracle.grid_tanh(12, H, 0.7)
    dt, tau_g = 0.4, 0.5
    c = oracle.Case3D(*n, walls=(False, False, True), thermal=True, dt=dt, tau=0.5, tau_g=tau_g,
                      T_bottom=0.5, T_top=-0.5, zf=zf)
    zc = 0.5 * (zf[1:] + zf[:-1])
    G = -1.0 / H
    s = (12, 4, 4)
    T = (0.5 + G * zc)[:, None, None] * np.ones(s)
    c.init(np.ones(s), np.zeros(s), np.zeros(s), np.zeros(s), T)
    c.g = W[:, None, None, None] * (T[None] - (tau_g + dt / 2) * C[:, 2][:, None, None, None] * G)
    c.step(50)
    np.testing.assert_allclose(c.moments()["T"], T, atol=1e-13)
    d = c.diagnostics()
    assert abs(d["nu_bottom"] - 1) < 1e-10 and abs(d["nu_top"] - 1) < 1e-10
