"""Steady Poiseuille accuracy (sec. 3.2, Figs. 3-5) through the library:
uniform-grid FV converges faster than ST (third against second order at
coarse resolution), wall-refined FV grids reach on a few cells the
accuracy ST needs many nodes for, and every run is accurate to the
Mach-number plateau."""
import sys

import pytest

from paper_1505_03271_amd import accuracy

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_poiseuille_orders_and_stretched_grids():
    e = {}
    for key in [("st", "uniform", 8), ("st", "uniform", 16), ("st", "uniform", 46), ("heun", "uniform", 8),
                ("heun", "uniform", 16), ("heun", "tanh", 8), ("heun", "tanh", 11), ("heun", "sinh", 8),
                ("heun", "chebyshev", 11)]:
        e[key] = accuracy.poiseuille_error(key[0], key[2], grid=key[1])[0]
        say(f"  {key}: {e[key]:.3e}")
    order_fv = e[("heun", "uniform", 8)] / e[("heun", "uniform", 16)]
    order_st = e[("st", "uniform", 8)] / e[("st", "uniform", 16)]
    assert order_fv > 8.0                 # at least third order from N = 8 to 16
    assert order_fv > order_st            # ST about second order
    # sec. 3.2: tanh with N = 11 about as accurate as ST with N ~ 46
    assert e[("heun", "tanh", 11)] < 2.0 * e[("st", "uniform", 46)]
    assert e[("heun", "tanh", 11)] < 0.5 * e[("st", "uniform", 16)]
    # every stretched grid at N = 8 beats the uniform FV grid at N = 8 by far
    for grid in ("tanh", "sinh"):
        assert e[("heun", grid, 8)] < 0.1 * e[("heun", "uniform", 8)]
    assert e[("heun", "chebyshev", 11)] < e[("st", "uniform", 16)] / 3.0
