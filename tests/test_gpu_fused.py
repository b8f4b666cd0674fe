"""Fused steps (the predictor and the corrector of a Heun step in one
launch, lb_set_fv_fused) against separate predictor and corrector launches:
bit-identical states for every storage format that has them (FP32
arithmetic), with and without walls, every item height (the ghost rows of
the second half at a bottom wall are written from rows 0 and 1 at every
position of an item), ragged widths, with renewed thermal references,
through captured graphs, and at the 4096^2 benchmark shape.  The separate
launches equal the oracle (FP64) and its bounds (narrower storage) in the
parity tests, so the fused steps do too; FP64 storage has no fused step (the
setting is accepted and the steps use separate launches)."""
import sys

import numpy as np
import pytest

import paper_1505_03271_amd as lb
import workloads
from gpu_common import make_pair, random_fields, rel_max

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(nx, ny, storage, thermal, wall_y, stretched=True, lanes=0, chunk=0, rebase=0):
    kw = dict(thermal=thermal, wall_y=wall_y, dt=0.35, tau=0.3, tau_g=0.4)
    if thermal:
        kw.update(beta_g=2e-5, T_bottom=0.2, T_top=-0.2)
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
    return sims


def _same(a, b, label):
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa, sb), f"{label}: fused and separate launches differ"
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16", "bf16s", "f16s"])
@pytest.mark.parametrize("thermal,wall_y", [(True, True), (True, False), (False, True), (False, False)])
def test_fused_equals_separate_launches(storage, thermal, wall_y):
    say(f"fused vs separate {storage} thermal={thermal} wall_y={wall_y}")
    for nx, ny, lanes in ((300, 77, 0), (300, 77, 256), (61, 40, 0), (530, 21, 256)):
        a, b = _pair(nx, ny, storage, thermal, wall_y, lanes=lanes)
        for n in (9, 1, 4):
            a.step(n)
            b.step(n)
        _same(a, b, f"{nx}x{ny} lanes {lanes}")


@pytest.mark.parametrize("storage", ["f32", "bf16s"])
@pytest.mark.parametrize("chunk", [1, 2, 3, 4, 5, 6, 7, 8, 12])
def test_fused_every_item_height(storage, chunk):
    """Heights below the second stage's reach put the wall images of rows
    0, 1 and ny-1, ny-2 at every position of an item."""
    say(f"fused item height {chunk} {storage}")
    a, b = _pair(90, 23, storage, True, True, chunk=chunk)
    a.step(6)
    b.step(6)
    _same(a, b, f"chunk {chunk}")


@pytest.mark.parametrize("storage,rebase", [("bf16s", 3), ("f32", 5), ("f16s", 1)])
def test_fused_with_renewed_references(storage, rebase):
    say(f"fused with rebase every {rebase} {storage}")
    a, b = _pair(200, 40, storage, True, True, rebase=rebase)
    for n in (11, 2, 7):
        a.step(n)
        b.step(n)
    _same(a, b, f"rebase {rebase}")


@pytest.mark.parametrize("storage", ["f16", "bf16s", "f32"])
def test_fused_through_captured_graphs(storage):
    """lb_step replays graphs of 32 steps (a predictor, 31 fused passes and a
    corrector each) around the rest of the steps."""
    say(f"fused graphs {storage}")
    a, b = _pair(150, 60, storage, True, True)
    for n in (70, 33, 64):
        a.step(n)
        b.step(n)
        a.sync()
        assert np.array_equal(a.get_state(), b.get_state()), f"after {n} more steps"
    a.close()
    b.close()


def test_fused_pass_is_used_and_f64_runs_separate_launches():
    """The kernel timing shows one fused launch per step for FP32 storage
    and none for FP64 storage, whose results still equal the oracle's."""
    nx, ny = 133, 46
    say("fused launches counted")
    kw = dict(thermal=True, wall_y=True, dt=0.35, tau=0.3, tau_g=0.4, beta_g=2e-5, T_bottom=0.2, T_top=-0.2)
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
    """rb4096 (4096^2, tanh(2.5), Ra = 1e10, BF16S): three steps fused and
    separate give the same bits."""
    say("fused at 4096^2")
    cfg = workloads.rb4096_config()
    n = cfg["nx"]
    kw = dict(thermal=True, wall_y=True, dt=cfg["dt"], tau=cfg["tau"], tau_g=cfg["tau_g"], beta_g=cfg["beta_g"],
              T0=cfg["T0"], T_bottom=cfg["T_bottom"], T_top=cfg["T_top"])
    states = []
    for fused in (1, 0):
        sim = lb.Sim(n, n, scheme="heun", storage="bf16s", stream=lb.current_stream(), **kw)
        sim.set_grid(cfg["xf"], cfg["yf"])
        sim.init(cfg["rho"], cfg["ux"], cfg["uy"], cfg["T"])
        sim.set_fv_fused(fused)
        sim.step(3)
        states.append(sim.get_state())
        sim.close()
    assert np.array_equal(states[0], states[1])


@pytest.mark.parametrize("storage,thermal,fused_by_default", [("f32", True, True), ("bf16s", True, True),
                                                              ("bf16s", False, False), ("f16", False, True)])
def test_automatic_setting(storage, thermal, fused_by_default):
    """The default (-1) uses fused steps where they measured faster: with
    thermal populations in every format, without them except for split
    storage; 1 forces them, 0 turns them off, other values are refused."""
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
