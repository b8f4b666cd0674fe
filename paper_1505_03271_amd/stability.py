"""Stability and viscosity measurements of the FV schemes on the decaying
Kolmogorov (shear-wave) flow of sec. 3.1 and sec. 4 (Fig. 6), run through
liblb on the GPU.

The flow lives on [L_x, L_y] = [1, 64] in the paper; the library needs at
least four cells per axis, so the domain here is 4 x n cells, periodic, with
u_x(y) = A sin(2 pi y / L_y).  A seeded 1e-6 perturbation of every mode lets
unstable modes grow.  With dims=1 (the paper's one-column set-up) the
perturbation depends on y only: every column then computes the same values,
so the state stays exactly x-independent and only y modes exist.  With
dims=2 it varies in x too, which seeds the two-dimensional modes, whose
stability limit is lower.

    from paper_1505_03271_amd import stability
    stability.dt_max("heun", 0.5)          # largest stable time step
    stability.viscosity("heun", 0.5, 1.0)  # measured nu / (tau cs^2)
"""
import math

import numpy as np

from . import Sim, current_stream, grid_uniform


def kolmogorov(scheme, tau, dt, n=64, amplitude=0.01, noise=1e-6, storage="f64", seed=3, stream=None, dims=1):
    """A Sim holding the decaying Kolmogorov flow (equilibrium start)."""
    sim = Sim(4, n, scheme=scheme, storage=storage, dt=dt, tau=tau,
              stream=stream if stream is not None else current_stream())
    sim.set_grid(grid_uniform(4, 4.0), grid_uniform(n, float(n)))
    r = np.random.default_rng(seed)
    y = np.arange(n) + 0.5
    cols = 4 if dims == 2 else 1
    ux = amplitude * np.sin(2 * math.pi * y / n)[:, None] + noise * r.standard_normal((n, cols))
    uy = noise * r.standard_normal((n, cols)) * np.ones((1, 4))
    sim.init(np.ones((n, 4)), ux * np.ones((1, 4)), uy)
    return sim


def is_stable(scheme, tau, dt, steps=3000, n=64, storage="f64", dims=1):
    """True when the kinetic energy stays finite and below its initial value
    over `steps` steps (a decaying flow only loses energy)."""
    sim = kolmogorov(scheme, tau, dt, n=n, storage=storage, dims=dims)
    try:
        e0 = sim.diagnostics()["ekin"]
        sim.step(steps)
        d = sim.diagnostics()
        e = d["ekin"]
        return d["nonfinite"] == 0.0 and math.isfinite(e) and e <= e0
    finally:
        sim.close()


def dt_max(scheme, tau, lo=0.02, hi=4.0, iters=12, steps=3000, n=64, storage="f64", dims=1):
    """Largest stable time step by bisection between lo (stable) and hi
    (unstable); returns (lo, hi) bracketing the limit after `iters` halvings
    of the interval (the ST scheme has dt = 1 fixed and is not a choice)."""
    if scheme == "st":
        raise ValueError("the ST step has dt = dx = 1")
    if not is_stable(scheme, tau, lo, steps, n, storage, dims):
        return 0.0, lo
    if is_stable(scheme, tau, hi, steps, n, storage, dims):
        return hi, math.inf
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if is_stable(scheme, tau, mid, steps, n, storage, dims):
            lo = mid
        else:
            hi = mid
    return lo, hi


def viscosity(scheme, tau, dt=1.0, n=64, amplitude=0.01, periods=0.5, samples=20, storage="f64"):
    """Measured kinematic viscosity over tau cs^2 (sec. 3.1): the kinetic
    energy of the shear wave decays as exp(-2 k^2 nu t), k = 2 pi / L_y; nu
    is the least-squares slope of log E over `samples` points spanning
    `periods` e-folding times of the amplitude."""
    cs2 = 1.0 / 3.0
    nu_th = tau * cs2
    k = 2 * math.pi / n
    if scheme == "st":
        dt = 1.0
    t_total = periods / (nu_th * k * k)
    every = max(1, int(round(t_total / dt / samples)))
    sim = kolmogorov(scheme, tau, dt, n=n, amplitude=amplitude, noise=0.0, storage=storage)
    try:
        t, logE = [], []
        for q in range(samples + 1):
            if q:
                sim.step(every)
            t.append(q * every * dt)
            logE.append(math.log(sim.diagnostics()["ekin"]))
        slope = np.polyfit(np.array(t[1:]), np.array(logE[1:]), 1)[0]
        return -slope / (2 * k * k) / nu_th
    finally:
        sim.close()
