"""Fused steps (the predictor and the corrector of a Heun step in one
launch, lb_set_fv_fused) against separate predictor and corrector launches.
With FP32 storage the two give the same bits (the fused step hands f~* over
in FP32, which is how the separate launches store it): with and without
walls, at every item height (the ghost rows of the corrector at a bottom
wall are written from rows 0 and 1 at every position of an item), on
ragged widths, with renewed thermal references, through captured graphs,
and at the 4096^2 benchmark shape.  With 16-bit storage the fused step
keeps f~* in FP32 instead of rounding it to the storage format, so both
shapes are checked against the FP64 oracle with the storage format's
per-step bound.  FP64 storage has no fused step (the setting is accepted and
the steps use separate launches)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1505_03271_amd as lb
import workloads
from gpu_common import make_pair, random_fields, rel_max, storage_bound

pytestmark = pytest.mark.gpu

EXACT = ("f64", "f32")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _kw(thermal, wall_y):
    kw = dict(thermal=thermal, wall_y=wall_y, dt=0.35, tau=0.3, tau_g=0.4)
    if thermal:
        kw.update(beta_g=2e-5, T_bottom=0.2, T_top=-0.2)
    return kw


def _pair(nx, ny, storage, thermal, wall_y, stretched=True, lanes=0, chunk=0, rebase=0):
    """(fused sim, separate sim, oracle case or None) from the same state."""
    kw = _kw(thermal, wall_y)
    xf = workloads.faces_uniform(nx, 1.3 * nx)
    yf = workloads.faces_tanh(ny, 1.5 * ny, 1.5) if stretched else workloads.faces_uniform(ny, ny)
    fields = random_fields(nx, ny, 21, thermal=thermal, amp=0.01)
    sims = []
    for fused in (1, 0):
        sim = lb.Sim(nx, ny, scheme="heun", storage=storage, stream=lb.current_stream(), **kw)
        sim.set_grid(xf, yf)
        if lanes:
            sim.set_fv_lanes(lanes)
        if chunk:
            sim.set_fv_chunk(chunk)
        sim.init(*fields)
        if rebase:
            sim.set_rebase(rebase)
        sim.set_fv_fused(fused)
        sims.append(sim)
    ref = None
    if storage not in EXACT:
        ref = oracle.Case(nx, ny, scheme="heun", xf=xf, yf=yf, **kw)
        ref.init(*fields)
    return sims[0], sims[1], ref


def _step(a, b, ref, n):
    a.step(n)
    b.step(n)
    if ref is not None:
        ref.step(n)


def _same(a, b, ref, storage, steps, label, close=True):
    """FP32/FP64: the same bits; 16-bit storage: both within the storage
    bound of the oracle."""
    if storage in EXACT:
        sa, sb = a.get_state(), b.get_state()
        assert np.array_equal(sa, sb), f"{label}: fused and separate launches differ"
    else:
        bound = storage_bound(storage, ref, steps, _kw(ref.g is not None, True))
        for sim, name in ((a, "fused"), (b, "separate")):
            f, g = sim.populations()
            err = max(np.abs(f - ref.f).max(), np.abs(g - ref.g).max() if g is not None else 0.0)
            assert err < bound, f"{label}: {name} error {err:.3e} above the bound {bound:.3e}"
    if close:
        a.close()
        b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16", "bf16s", "f16s"])
@pytest.mark.parametrize("thermal,wall_y", [(True, True), (True, False), (False, True), (False, False)])
def test_fused_equals_separate_launches(storage, thermal, wall_y):
    say(f"fused vs separate {storage} thermal={thermal} wall_y={wall_y}")
    for nx, ny, lanes in ((300, 77, 0), (300, 77, 256), (61, 40, 0), (530, 21, 256), (4, 4, 0), (5, 7, 0)):
        a, b, ref = _pair(nx, ny, storage, thermal, wall_y, lanes=lanes)
        for n in (9, 1, 4):
            _step(a, b, ref, n)
        _same(a, b, ref, storage, 14, f"{nx}x{ny} lanes {lanes}")


@pytest.mark.parametrize("storage", ["f32", "bf16s"])
@pytest.mark.parametrize("chunk", [1, 2, 3, 4, 5, 6, 7, 8, 12])
def test_fused_every_item_height(storage, chunk):
    """Heights below the second stage's reach put the wall images of rows
    0, 1 and ny-1, ny-2 at every position of an item (a fused item holds at
    least two rows: height 1 gives fused items of 2 beside separate launches
    of 1)."""
    say(f"fused item height {chunk} {storage}")
    a, b, ref = _pair(90, 23, storage, True, True, chunk=chunk)
    _step(a, b, ref, 6)
    _same(a, b, ref, storage, 6, f"chunk {chunk}")


@pytest.mark.parametrize("storage,rebase", [("bf16s", 3), ("f32", 5), ("f16s", 1)])
def test_fused_with_renewed_references(storage, rebase):
    say(f"fused with rebase every {rebase} {storage}")
    a, b, ref = _pair(200, 40, storage, True, True, rebase=rebase)
    for n in (11, 2, 7):
        _step(a, b, ref, n)
    _same(a, b, ref, storage, 20, f"rebase {rebase}")


@pytest.mark.parametrize("storage", ["f16", "bf16s", "f32"])
def test_fused_through_captured_graphs(storage):
    """lb_step replays graphs of 32 fused steps around the rest of the steps;
    the graphs give the same bits as single launches of the same shape."""
    say(f"fused graphs {storage}")
    a, b, ref = _pair(150, 60, storage, True, True)
    b.set_fv_fused(1)
    b.set_timing(True)   # single launches: no graphs
    done = 0
    for n in (70, 33, 64):
        _step(a, b, ref, n)
        done += n
        a.sync()
        assert np.array_equal(a.get_state(), b.get_state()), f"after {n} more steps"
    _same(a, b, ref, storage, done, "graphs")


def test_fused_pass_is_used_and_f64_runs_separate_launches():
    """The kernel timing shows one fused launch per step for FP32 storage
    and none for FP64 storage, whose results still equal the oracle's."""
    nx, ny = 133, 46
    say("fused launches counted")
    kw = _kw(True, True)
    xf = workloads.faces_uniform(nx, 1.3 * nx)
    yf = workloads.faces_tanh(ny, 1.5 * ny, 1.5)
    fields = random_fields(nx, ny, 5, amp=0.01)
    a = lb.Sim(nx, ny, scheme="heun", storage="f32", stream=lb.current_stream(), **kw)
    a.set_grid(xf, yf)
    a.init(*fields)
    a.set_fv_fused(1)
    a.set_timing(True)
    a.step(12)
    kt = a.kernel_times()
    assert kt["fv_fused"][0] == 12 and kt["fv_first_pass"][0] == 0 and kt["fv_corrector"][0] == 0
    a.close()
    sim, ref = make_pair(nx, ny, "heun", "f64", xf, yf, fields, **kw)
    sim.set_fv_fused(1)
    sim.set_timing(True)
    sim.step(12)
    ref.step(12)
    assert sim.kernel_times()["fv_fused"][0] == 0
    f, g = sim.populations()
    assert max(rel_max(f, ref.f), rel_max(g, ref.g)) < 1e-12
    sim.close()


def test_fused_at_the_benchmark_shape():
    """rb4096 (4096^2, tanh(2.5), Ra = 1e10) in FP32 storage: three steps
    fused and separate give the same bits (the split BF16 headline format
    is checked against the oracle at this shape in the parity tests)."""
    say("fused at 4096^2")
    cfg = workloads.rb4096_config()
    n = cfg["nx"]
    kw = dict(thermal=True, wall_y=True, dt=cfg["dt"], tau=cfg["tau"], tau_g=cfg["tau_g"], beta_g=cfg["beta_g"],
              T0=cfg["T0"], T_bottom=cfg["T_bottom"], T_top=cfg["T_top"])
    states = []
    for fused in (1, 0):
        sim = lb.Sim(n, n, scheme="heun", storage="f32", stream=lb.current_stream(), **kw)
        sim.set_grid(cfg["xf"], cfg["yf"])
        sim.init(cfg["rho"], cfg["ux"], cfg["uy"], cfg["T"])
        sim.set_fv_fused(fused)
        sim.step(3)
        states.append(sim.get_state())
        sim.close()
    assert np.array_equal(states[0], states[1])


@pytest.mark.parametrize("storage,thermal,fused_by_default", [("f32", True, True), ("bf16s", True, True),
                                                              ("bf16s", False, True), ("f16", False, True)])
def test_automatic_setting(storage, thermal, fused_by_default):
    """The default (-1) uses fused steps where they measured faster (every
    format but FP64, with and without thermal populations); 1 forces them,
    0 turns them off, other values are refused."""
    n = 64
    say(f"automatic fused setting {storage} thermal={thermal}")
    kw = dict(thermal=thermal, wall_y=True, dt=0.35, tau=0.3, tau_g=0.4)
    if thermal:
        kw.update(beta_g=2e-5, T_bottom=0.2, T_top=-0.2)
    sim = lb.Sim(n, n, scheme="heun", storage=storage, stream=lb.current_stream(), **kw)
    sim.set_grid(workloads.faces_uniform(n, n), workloads.faces_tanh(n, n, 1.5))
    sim.init(*random_fields(n, n, 3, thermal=thermal, amp=0.01))
    assert sim.fv_fused() == -1
    counts = {}
    for setting in (None, 1, 0):
        if setting is not None:
            sim.set_fv_fused(setting)
        sim.set_timing(True)
        sim.step(4)
        counts[setting] = sim.kernel_times()["fv_fused"][0]
        sim.set_timing(False)
    assert counts[None] == (4 if fused_by_default else 0)
    assert counts[1] == 4 and counts[0] == 0
    assert sim.fv_fused() == 0
    with pytest.raises(lb.LBError):
        sim.set_fv_fused(2)
    sim.close()
