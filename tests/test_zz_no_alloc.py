"""lb_diagnostics_noalloc (the diagnostics for callers that cannot allocate:
its partial sums live in the library's static device array) against
lb_diagnostics on the same state, through the C ABI: two calls in a row,
the second on a smaller grid (fewer partial sums than the first left in the
shared array), and a call captured in a HIP graph by the caller."""
import sys

import numpy as np
import pytest

import paper_1505_03271_amd as lb
import workloads

pytestmark = pytest.mark.gpu

KEYS = ["mass", "ekin", "etherm", "nu_bottom", "nu_top", "nu_vol", "volume", "nonfinite"]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rb(n_x, n_y, storage, seed, steps):
    P = workloads.rb_params(1e6, 1.0, n_x, n_y, aspect=n_x / n_y, stretch=2.0)
    rho, ux, uy, T = workloads.rb_fields(n_x, P["yf"], P["dT"], P["T0"], P["beta_g"], seed_index=seed)
    sim = lb.Sim(n_x, n_y, scheme="heun", storage=storage, thermal=True, wall_y=True, dt=P["dt"], tau=P["tau"],
                 tau_g=P["tau_g"], beta_g=P["beta_g"], T0=P["T0"], T_bottom=P["T_bottom"], T_top=P["T_top"],
                 stream=lb.current_stream())
    sim.set_grid(P["xf"], P["yf"])
    sim.init(rho, ux, uy, T)
    sim.step(steps)
    return sim


def _check(got, want, label):
    ref = np.array([want[k] for k in KEYS])
    say(f"  {label}: {got}")
    assert np.all(np.isfinite(got)), label
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-300, err_msg=label)


@pytest.mark.parametrize("storage", ["f64", "bf16s", "f32"])
def test_noalloc_diagnostics_equal_lb_diagnostics(storage):
    import torch
    say(f"noalloc diagnostics {storage}")
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    big = _rb(1100, 300, storage, 3, 40)        # 330 000 cells: all 1024 partial sums
    small = _rb(96, 40, storage, 4, 25)         # 3 840 cells: 15 partial sums
    for sim, label in ((big, "1100x300"), (small, "96x40"), (big, "1100x300 again")):
        sim.diagnostics_noalloc(out.data_ptr())
        torch.cuda.synchronize()
        _check(out.cpu().numpy(), sim.diagnostics(), label)
        out.fill_(float("nan"))
    big.close()
    small.close()


def test_noalloc_diagnostics_inside_a_captured_graph():
    """A caller captures steps and the diagnostics in one graph of its own:
    the call allocates nothing and does not synchronise, so it can be
    captured; every replay's output equals lb_diagnostics of a simulation
    stepped the same number of times without a graph (with eager work and
    synchronisations between the replays)."""
    import ctypes
    import torch
    say("noalloc diagnostics under the caller's graph capture")
    side = torch.cuda.Stream()
    sim = _rb(200, 120, "bf16s", 5, 0)
    ref = _rb(200, 120, "bf16s", 5, 0)
    # a handle bound to the side stream, with the same state
    P = workloads.rb_params(1e6, 1.0, 200, 120, aspect=200 / 120, stretch=2.0)
    cap = lb.Sim(200, 120, scheme="heun", storage="bf16s", thermal=True, wall_y=True, dt=P["dt"], tau=P["tau"],
                 tau_g=P["tau_g"], beta_g=P["beta_g"], T0=P["T0"], T_bottom=P["T_bottom"], T_top=P["T_top"],
                 stream=ctypes.c_void_p(side.cuda_stream))
    cap.set_grid(P["xf"], P["yf"])
    cap.set_state(sim.get_state())
    sim.close()
    cap.step(1)                      # launch shape chosen before capture
    ref.step(1)
    torch.cuda.synchronize()
    out = torch.zeros((8,), dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        cap.step(4)
        cap.diagnostics_noalloc(out.data_ptr())
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        ref.step(4)
        _check(out.cpu().numpy(), ref.diagnostics(), f"replay {k}")
        out.fill_(float("nan"))      # eager work between the replays
        torch.cuda.synchronize()
    cap.close()
    ref.close()
