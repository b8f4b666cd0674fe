"""lb_step replays captured graphs of whole blocks of steps: the results
must be bit-identical to the same steps launched one by one (the timed path
launches every kernel itself), over several calls with other work and
synchronisations between the replays, for every scheme, with the buffer
swaps of the single-pass schemes and a rebase schedule that does not divide
the graph length."""
import sys

import numpy as np
import pytest

import paper_1505_03271_amd as lb
import workloads
from gpu_common import random_fields

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [("heun", "f64", 0), ("heun", "bf16s", 10), ("heun", "f32", 7), ("semi", "f32", 0), ("euler", "bf16", 0),
         ("st", "bf16", 0), ("st", "f32", 5)]


def _sim(scheme, storage, rebase, nx, ny):
    kw = dict(thermal=True, wall_y=True, tau=0.3, tau_g=0.4, beta_g=2e-5, T_bottom=0.2, T_top=-0.2)
    if scheme != "st":
        kw["dt"] = 0.1 if scheme == "euler" else 0.4   # within each scheme's stability limit
        xf, yf = workloads.faces_uniform(nx, nx), workloads.faces_tanh(ny, 2.0 * ny, 1.5)
    else:
        xf, yf = workloads.faces_uniform(nx, nx), workloads.faces_uniform(ny, ny)
    sim = lb.Sim(nx, ny, scheme=scheme, storage=storage, stream=lb.current_stream(), **kw)
    sim.set_grid(xf, yf)
    sim.init(*random_fields(nx, ny, 12, amp=0.01))
    if rebase:
        sim.set_rebase(rebase)
    return sim


@pytest.mark.parametrize("scheme,storage,rebase", CASES)
def test_graph_steps_equal_single_launches(scheme, storage, rebase):
    nx, ny = 70, 36
    say(f"step graphs {scheme} {storage} rebase {rebase}")
    direct = _sim(scheme, storage, rebase, nx, ny)
    direct.set_timing(True)          # every launch by the host
    graph = _sim(scheme, storage, rebase, nx, ny)
    for n in (70, 33, 64, 5, 96):
        direct.step(n)
        graph.step(n)
        m = graph.moments()          # other work and a synchronisation between replays
        assert np.all(np.isfinite(m["rho"]))
        assert np.array_equal(graph.get_state(), direct.get_state()), f"after {n} more steps"
    direct.close()
    graph.close()


def test_graphs_follow_a_new_grid_and_launch_shape():
    """The calls that change what the captured launches hold (grid, item
    height, item width) take effect in the next steps."""
    nx, ny = 300, 40
    say("step graphs after changes")
    a = _sim("heun", "f32", 0, nx, ny)
    b = _sim("heun", "f32", 0, nx, ny)
    b.set_timing(True)
    for sim in (a, b):
        sim.step(40)
        sim.set_fv_chunk(8)
        sim.step(40)
        sim.set_fv_lanes(64)
        sim.step(40)
        sim.set_grid(workloads.faces_uniform(nx, nx), workloads.faces_uniform(ny, ny))
        sim.step(40)
    assert np.array_equal(a.get_state(), b.get_state())
    a.close()
    b.close()
