"""The 3D (D3Q19) FV step through lb3_* against the 3D oracle: FP64 parity
at 1e-12 for the three schemes on stretched grids with walls and periodic
axes (thermal, isothermal), FP32 within its rounding bound, and the
conductive state as an exact steady state (Nu = 1)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1505_03271_amd as lb
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _fields(n, seed, thermal=True, amp=0.03):
    r = np.random.default_rng(seed)
    nx, ny, nz = n
    s = (nz, ny, nx)
    out = [1.0 + 0.01 * r.standard_normal(s)] + [amp * r.standard_normal(s) for _ in range(3)]
    out.append(0.3 * r.uniform(-1, 1, s) if thermal else None)
    return out


def _pair(n, scheme, storage, walls, thermal, faces, **kw):
    import torch
    sim = lb.Sim3(*n, scheme=scheme, storage=storage, thermal=thermal, walls=walls, stream=lb.current_stream(), **kw)
    sim.set_grid(*faces)
    ref = oracle.Case3D(*n, scheme=scheme, walls=walls, thermal=thermal, xf=faces[0], yf=faces[1], zf=faces[2], **kw)
    fields = _fields(n, sum(n), thermal)
    sim.init(*fields)
    ref.init(*fields)
    torch.cuda.synchronize()
    return sim, ref


CASES = [
    dict(id="thermal-zwalls", n=(37, 12, 18), walls=(False, False, True), thermal=True),
    dict(id="thermal-allwalls", n=(9, 14, 11), walls=(True, True, True), thermal=True),
    dict(id="isothermal-periodic", n=(20, 9, 7), walls=(False, False, False), thermal=False),
]


@pytest.mark.parametrize("case", CASES, ids=[c["id"] for c in CASES])
@pytest.mark.parametrize("scheme", ["heun", "semi", "euler"])
def test_fv3d_fp64_parity(case, scheme):
    n, walls, thermal = case["n"], case["walls"], case["thermal"]
    say(f"3D {scheme} f64 {case['id']} {n}")
    r = np.random.default_rng(5)
    faces = [np.concatenate([[0.0], np.cumsum(r.uniform(0.6, 1.4, k))]) if w else np.arange(k + 1.0)
             for k, w in zip(n, walls)]
    faces[2] = workloads.faces_tanh(n[2], 2.0 * n[2], 1.2) if walls[2] else faces[2]
    dt = {"heun": 0.4, "semi": 0.2, "euler": 0.1}[scheme]
    kw = dict(dt=dt, tau=0.3, tau_g=0.25, a=(2e-5, -1e-5, 3e-5), beta_g=1e-3 if thermal else 0.0, T0=0.05,
              T_bottom=0.5, T_top=-0.5)
    sim, ref = _pair(n, scheme, "f64", walls, thermal, faces, **kw)
    sim.step(12)
    ref.step(12)
    f, g = sim.populations()
    assert np.abs(f - ref.f).max() < 1e-12 * np.abs(ref.f).max()
    if thermal:
        assert np.abs(g - ref.g).max() < 1e-12 * np.abs(ref.g).max()
    d, od = sim.diagnostics(), ref.diagnostics()
    assert abs(d["mass"] - od["mass"]) < 1e-12 * od["mass"]
    if thermal and walls[2]:
        for key in ("nu_bottom", "nu_top"):
            assert abs(d[key] - od[key]) < 1e-9, key


def test_fv3d_fp32_against_oracle():
    n, walls = (37, 12, 18), (False, False, True)
    say("3D heun f32")
    faces = [np.arange(38.0), np.arange(13.0), workloads.faces_tanh(18, 36.0, 1.2)]
    kw = dict(dt=0.4, tau=0.3, tau_g=0.25, beta_g=1e-3, T0=0.05, T_bottom=0.5, T_top=-0.5)
    sim, ref = _pair(n, "heun", "f32", walls, True, faces, **kw)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None, None, None]
    for steps in (1, 5):
        sim.step(1 if steps == 1 else 4)
        ref.step(1 if steps == 1 else 4)
        f, g = sim.populations()
        so = max(np.abs(ref.f - w).max(), np.abs(ref.g).max())
        bound = steps * (8 * 2.0 ** -24 * so + 64 * 2.0 ** -24)
        ef, eg = np.abs(f - ref.f).max(), np.abs(g - ref.g).max()
        say(f"  steps={steps} err f={ef:.3e} g={eg:.3e} bound={bound:.3e}")
        assert ef < bound and eg < bound


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_fv3d_conduction_steady(storage):
    n = (8, 6, 16)
    H = 32.0
    zf = workloads.faces_tanh(16, H, 1.2)
    dt, tau_g = float(np.diff(zf).min()), 0.5
    sim = lb.Sim3(*n, scheme="heun", storage=storage, thermal=True, walls=(False, False, True), dt=dt, tau=0.5,
                  tau_g=tau_g, T_bottom=0.5, T_top=-0.5, stream=lb.current_stream())
    sim.set_grid(np.arange(9.0), np.arange(7.0), zf)
    zc = 0.5 * (zf[1:] + zf[:-1])
    T = (0.5 - zc / H)[:, None, None] * np.ones((16, 6, 8))
    # a conductive start from equilibrium populations: the missing flux part of
    # g relaxes, and its trace diffuses out within three diffusion times H^2 / kappa
    sim.init(np.ones((16, 6, 8)), np.zeros((16, 6, 8)), np.zeros((16, 6, 8)), np.zeros((16, 6, 8)), T)
    sim.step(int(3 * H * H / (tau_g / 3) / dt))
    d = sim.diagnostics()
    tol = 1e-9 if storage == "f64" else 2e-4
    assert abs(d["nu_bottom"] - 1) < tol and abs(d["nu_top"] - 1) < tol and abs(d["nu_vol"] - 1) < tol


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("walls,thermal", [((False, False, True), True), ((True, True, True), True),
                                          ((True, False, False), False)])
def test_fv3d_tiled_and_per_cell_updates_are_bit_identical(storage, walls, thermal):
    """The LDS-tiled flux + update kernel (32 x 4 x 4 tiles) against the
    per-cell one on grids that span several tiles with ragged edges on every
    axis: same operations in the same order, so the same bits."""
    n = (70, 13, 9)
    say(f"3D tiled vs per-cell {storage} walls={walls} thermal={thermal}")
    r = np.random.default_rng(17)
    faces = [np.concatenate([[0.0], np.cumsum(r.uniform(0.7, 1.3, k))]) for k in n]
    kw = dict(dt=0.4, tau=0.3, tau_g=0.25, a=(2e-5, -1e-5, 3e-5), beta_g=1e-3 if thermal else 0.0, T0=0.05,
              T_bottom=0.5, T_top=-0.5)
    out = {}
    for kind in ("tiled", "gather"):
        sim = lb.Sim3(*n, scheme="heun", storage=storage, thermal=thermal, walls=walls, stream=lb.current_stream(),
                      **kw)
        sim.set_update(kind)
        sim.set_grid(*faces)
        sim.init(*_fields(n, 3, thermal))
        sim.step(6)
        out[kind] = sim.populations()
        sim.close()
    for a, b in zip(out["tiled"], out["gather"]):
        if a is not None:
            assert np.array_equal(a, b)


def test_fv3d_benchmark_shape_tiled_equals_per_cell():
    """The benchmark's 3D workload and launch shape (256^3 thermal RB, FP32,
    tanh z grid; tiles dealt to XCDs in z columns): two Heun steps with the
    tiled update and with the per-cell update give the same moments bit for
    bit and the same FP64 diagnostics."""
    cfg = workloads.rb3d_config(256, 1e8, 2.0)
    say("3D 256^3 tiled vs per-cell")
    out = {}
    for kind in ("tiled", "gather"):
        sim = lb.Sim3(256, 256, 256, scheme="heun", storage="f32", thermal=True, walls=(False, False, True),
                      dt=cfg["dt"], tau=cfg["tau"], tau_g=cfg["tau_g"], beta_g=cfg["beta_g"], T0=cfg["T0"],
                      T_bottom=cfg["T_bottom"], T_top=cfg["T_top"], stream=lb.current_stream())
        sim.set_update(kind)
        sim.set_grid(cfg["xf"], cfg["yf"], cfg["zf"])
        sim.init(cfg["rho"], cfg["ux"], cfg["uy"], cfg["uz"], cfg["T"])
        sim.step(2)
        out[kind] = (sim.moments(), sim.diagnostics())
        sim.close()
    (mt, dt_), (mg, dg) = out["tiled"], out["gather"]
    for k in mt:
        assert np.array_equal(mt[k], mg[k]), k
    assert dt_ == dg
    assert dt_["nonfinite"] == 0
