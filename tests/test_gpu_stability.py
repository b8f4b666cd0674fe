"""Stability map and viscosity of the FV schemes (sec. 3.1 and sec. 4,
Fig. 6) measured through liblb on the decaying Kolmogorov flow, against the
oracle's decisions and the paper's statements."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1505_03271_amd import stability

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_stable(scheme, tau, dt, steps=3000, n=64, dims=1):
    c = oracle.Case(4, n, scheme=scheme, dt=dt, tau=tau, xf=np.arange(5.0), yf=np.arange(n + 1.0))
    r = np.random.default_rng(3)
    y = np.arange(n) + 0.5
    cols = 4 if dims == 2 else 1
    ux = 0.01 * np.sin(2 * math.pi * y / n)[:, None] + 1e-6 * r.standard_normal((n, cols))
    uy = 1e-6 * r.standard_normal((n, cols)) * np.ones((1, 4))
    c.init(np.ones((n, 4)), ux * np.ones((1, 4)), uy)
    e0 = c.diagnostics()["ekin"]
    c.step(steps)
    d = c.diagnostics()
    return d["nonfinite"] == 0.0 and math.isfinite(d["ekin"]) and d["ekin"] <= e0


@pytest.mark.parametrize("scheme,tau,dt,dims", [("heun", 0.5, 1.6, 1), ("heun", 0.5, 1.9, 1), ("semi", 0.2, 0.9, 1),
                                                ("euler", 0.25, 0.45, 1), ("euler", 0.25, 0.55, 1),
                                                ("heun", 0.5, 0.9, 2), ("heun", 0.5, 1.0, 2)])
def test_stability_decision_matches_oracle(scheme, tau, dt, dims):
    say(f"stability {scheme} tau={tau} dt={dt} dims={dims}")
    assert stability.is_stable(scheme, tau, dt, dims=dims) == _oracle_stable(scheme, tau, dt, dims=dims)


def test_stability_map_statements_of_the_paper():
    """On the paper's one-column Kolmogorov flow (sec. 4, Fig. 6): Heun has
    dt_max > 1 for tau > 1/8 and about 1.7 near tau = 1/2; Euler is bounded
    by 2 tau; the semi-implicit scheme alone stays below Heun.  Modes that
    vary along x (a 4-column domain seeded in x too) lower the Heun limit
    below 1."""
    out = {}
    for scheme, taus in (("heun", (0.15, 0.25, 0.5, 1.0)), ("semi", (0.15, 0.5)), ("euler", (0.15, 0.5))):
        for tau in taus:
            lo, hi = stability.dt_max(scheme, tau, iters=9)
            out[(scheme, tau)] = lo
            say(f"  dt_max {scheme} tau={tau}: [{lo:.3f}, {hi:.3f}]")
    for tau in (0.15, 0.25, 0.5, 1.0):
        assert out[("heun", tau)] > 1.0
    assert out[("heun", 0.5)] > 1.4
    lo2, hi2 = stability.dt_max("heun", 0.5, iters=9, dims=2)
    say(f"  dt_max heun tau=0.5, x-varying modes: [{lo2:.3f}, {hi2:.3f}]")
    assert lo2 < out[("heun", 0.5)]
    for tau in (0.15, 0.5):
        assert out[("euler", tau)] <= 2 * tau * 1.01
        assert out[("semi", tau)] < out[("heun", tau)]


def test_viscosity_error_fv_and_st():
    """sec. 3.1: the measured viscosity approaches tau cs^2; at tau = 1/2
    both schemes are accurate and ST is the more accurate one."""
    res = {}
    for scheme in ("heun", "st"):
        for tau in (0.2, 0.5, 1.0):
            res[(scheme, tau)] = stability.viscosity(scheme, tau, dt=1.0) - 1.0
            say(f"  nu error {scheme} tau={tau}: {res[(scheme, tau)]:+.3e}")
    assert abs(res[("heun", 0.5)]) < 0.02 and abs(res[("st", 0.5)]) < 0.02
    assert abs(res[("st", 0.5)]) < abs(res[("heun", 0.5)])
