"""Steady Poiseuille accuracy of the FV and ST steps (sec. 3.2, Figs. 3-5),
run through liblb on the GPU.

A channel of width L between no-slip walls (y = 0, L), periodic along x,
driven by a constant acceleration a_x = 8 nu U / L^2 so that the analytic
profile U(y) = 4 U y (L - y) / L^2 is the steady state; Re = L U / nu.  The
flow starts from that profile and runs for `visc_times` viscous times L^2/nu;
the error is the relative L2 difference of the computed u_x(y) from U(y) at
the cell centres, ||u - U||_2 / ||U||_2 with ||f||_2^2 = sum f_i^2 dy_i.

FV (any grid): N cells on [0, L] (lattice units with the mean cell L / N),
nu = U L / Re, dt = cfl x the smallest cell.  ST: N nodes with dx = dt = 1,
so the same physical flow at the same Mach number has nu = U N / Re in its
own lattice units.

    from paper_1505_03271_amd import accuracy
    accuracy.poiseuille_error("heun", 11, grid="tanh")
"""
import math

import numpy as np

from . import Sim, current_stream, grid_chebyshev, grid_sinh, grid_tanh, grid_uniform

CS2 = 1.0 / 3.0
S1_TANH = 0.98   # the paper's stretching factors (sec. 3.2)
S2_SINH = 6.5


def faces(grid, n, L):
    if grid == "uniform":
        return grid_uniform(n, L)
    if grid == "tanh":
        return grid_tanh(n, L, math.atanh(S1_TANH))
    if grid == "sinh":
        return grid_sinh(n, L, S2_SINH)
    if grid == "chebyshev":
        return grid_chebyshev(n, L)
    raise ValueError(grid)


def poiseuille_error(scheme, n, grid="uniform", L=64.0, Re=10.0, U=0.05, cfl=1.0, visc_times=3.0,
                     storage="f64", stream=None):
    """Relative L2 error of the steady profile; returns (error, dict of the
    run's parameters)."""
    if scheme == "st":
        if grid != "uniform":
            raise ValueError("ST runs on the uniform unit grid")
        Ll, dt = float(n), 1.0
    else:
        Ll = L
    nu = U * Ll / Re
    yf = faces("uniform", n, Ll) if scheme == "st" else faces(grid, n, Ll)
    dy = np.diff(yf)
    if scheme != "st":
        dt = cfl * float(dy.min())
    ax = 8.0 * nu * U / (Ll * Ll)
    sim = Sim(4, n, scheme=scheme, storage=storage, wall_y=True, dt=dt, tau=nu / CS2, ax=ax,
              stream=stream if stream is not None else current_stream())
    try:
        sim.set_grid(grid_uniform(4, 4.0) if scheme == "st" else grid_uniform(4, 4.0 * float(dy.max())), yf)
        yc = 0.5 * (yf[1:] + yf[:-1])
        prof = 4.0 * U * yc * (Ll - yc) / (Ll * Ll)
        sim.init(np.ones((n, 4)), np.repeat(prof[:, None], 4, axis=1), np.zeros((n, 4)))
        steps = int(math.ceil(visc_times * Ll * Ll / nu / dt))
        sim.step(steps)
        ux = sim.moments()["ux"][:, 0]
        err = math.sqrt(float(np.sum((ux - prof) ** 2 * dy)) / float(np.sum(prof ** 2 * dy)))
        return err, dict(n=n, grid=grid, dt=dt, tau=nu / CS2, steps=steps, Ma=U / math.sqrt(CS2))
    finally:
        sim.close()
