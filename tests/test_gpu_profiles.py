"""Row profiles (lb_profiles): x averages of T, T^2, u_x^2, u_y^2, u_y T and
the height-dependent Nusselt number Nu(y) of sec. 5, against the same
definitions evaluated on the oracle's FP64 moments."""
import sys

import numpy as np
import pytest

import paper_1505_03271_amd as lb
import workloads
from gpu_common import make_pair, random_fields

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _expected(m, xf, yf, T_bottom, T_top, tau_g):
    w = np.diff(xf) / (xf[-1] - xf[0])
    avg = lambda a: (a * w[None, :]).sum(axis=1)
    Tm = avg(m["T"])
    out = dict(T_mean=Tm, T_rms=np.sqrt(np.maximum(avg(m["T"] ** 2) - Tm ** 2, 0.0)),
               ux_rms=np.sqrt(avg(m["ux"] ** 2)), uy_rms=np.sqrt(avg(m["uy"] ** 2)), uyT=avg(m["uy"] * m["T"]))
    yc = 0.5 * (yf[1:] + yf[:-1])
    ny = len(yc)
    H, kappa, dT = yf[-1] - yf[0], tau_g / 3.0, T_bottom - T_top
    nu = np.empty(ny)
    for j in range(ny):
        if j == 0:
            xs, vs = [yf[0], yc[0], yc[1]], [T_bottom, Tm[0], Tm[1]]
        elif j == ny - 1:
            xs, vs = [yc[-2], yc[-1], yf[-1]], [Tm[-2], Tm[-1], T_top]
        else:
            xs, vs = yc[j - 1:j + 2], Tm[j - 1:j + 2]
        c2, c1, _ = np.polyfit(np.asarray(xs) - yc[j], vs, 2)   # derivative at yc[j] = c1
        nu[j] = (out["uyT"][j] - kappa * c1) / (kappa * dT / H)
    out["Nu"] = nu
    return out


def test_profiles_fp64_against_oracle_moments():
    nx, ny = 300, 77
    say("profiles f64")
    r = np.random.default_rng(31)
    xf = np.concatenate([[0.0], np.cumsum(r.uniform(0.6, 1.4, nx))])
    yf = workloads.faces_tanh(ny, 2.0 * ny, 1.5)
    kw = dict(thermal=True, wall_y=True, dt=0.5, tau=0.3, tau_g=0.25, beta_g=1e-3, T_bottom=0.5, T_top=-0.5)
    sim, ref = make_pair(nx, ny, "heun", "f64", xf, yf, random_fields(nx, ny, 41), chunk=16, **kw)
    sim.step(10)
    ref.step(10)
    got = sim.profiles()
    exp = _expected(ref.moments(), xf, yf, 0.5, -0.5, 0.25)
    for key, e in exp.items():
        scale = max(np.abs(e).max(), 1e-300)
        # Nu(y) divides a difference of O(1) temperatures by kappa dT / H
        tol = 1e-9 if key == "Nu" else 1e-12
        assert np.abs(got[key] - e).max() <= tol * scale, key


@pytest.mark.parametrize("storage", ["f64", "bf16s"])
def test_conduction_nusselt_profile_is_one(storage):
    """The linear conductive state with the wall temperatures is an exact
    steady state; its Nu(y) is 1 at every height."""
    nx, ny = 64, 48
    say(f"conduction Nu(y) {storage}")
    H = 96.0
    yf = workloads.faces_tanh(ny, H, 1.5)
    xf = workloads.faces_uniform(nx, 64.0)
    tau_g, dt = 0.5, float(np.diff(yf).min())
    sim = lb.Sim(nx, ny, scheme="heun", storage=storage, thermal=True, wall_y=True, dt=dt, tau=0.5,
                 tau_g=tau_g, T_bottom=0.5, T_top=-0.5, stream=lb.current_stream())
    sim.set_grid(xf, yf)
    yc = 0.5 * (yf[1:] + yf[:-1])
    G = -1.0 / H
    T = np.repeat((0.5 + G * yc)[:, None], nx, axis=1)
    sim.init(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), T)
    # the steady populations carry the conductive flux: g = w (T - (tau_g + dt/2) c_y dT/dy)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])[:, None, None]
    g = w * (T[None] - (tau_g + dt / 2) * cy * G)
    f, _ = sim.populations()
    sim.set_populations(f, g)
    sim.step(200)
    p = sim.profiles()
    tol = 1e-10 if storage == "f64" else 2e-4
    assert np.abs(p["Nu"] - 1.0).max() < tol
    assert np.abs(p["T_mean"] - (0.5 + G * yc)).max() < (1e-12 if storage == "f64" else 1e-6)
    assert p["T_rms"].max() < (1e-7 if storage == "f64" else 1e-3)
