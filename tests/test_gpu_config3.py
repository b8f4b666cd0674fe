"""Rayleigh-Benard Ra = 1e8, Pr = 1, 1024 x 1024, tanh(2.0) wall refinement
(the seeded rb1024 workload: conductive start, hydrostatic density, +-1e-3
temperature noise), 500 steps of the semi-implicit + Heun scheme (eq:semi-heun),
in every storage format against the FP64 oracle run of the same steps.

500 steps is the horizon over which pointwise parity is meaningful for a
flow that becomes chaotic.  FP64 storage must equal the oracle to 1e-12;
FP32 arithmetic with FP32, split bfloat16 or split half storage must keep
the wall and volume Nusselt numbers within 1%; every format's relative L2
errors of the T and u fields and of the Nusselt numbers are printed (plain
bfloat16 offsets, which stagnate under this small time step, only
reported).  The split bfloat16 format is run with and without renewed
thermal references (lb_set_rebase) to show whether it needs them here."""
import sys
import threading
import time

import numpy as np
import pytest

import oracle
import paper_1505_03271_amd as lb
import workloads

pytestmark = pytest.mark.gpu

STEPS = 500


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _kw(cfg):
    return dict(thermal=True, wall_y=True, dt=cfg["dt"], tau=cfg["tau"], tau_g=cfg["tau_g"], beta_g=cfg["beta_g"],
                T0=cfg["T0"], T_bottom=cfg["T_bottom"], T_top=cfg["T_top"])


def _l2(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2) / np.mean(b ** 2)))


@pytest.mark.timeout(600)
def test_rb1024_500_steps_every_storage_against_the_oracle():
    cfg = workloads.rb1024_config()
    n = cfg["nx"]
    fields = (cfg["rho"], cfg["ux"], cfg["uy"], cfg["T"])
    # the oracle steps on the host cores while the GPU runs the formats
    ref = oracle.Case(n, n, scheme="heun", xf=cfg["xf"], yf=cfg["yf"], **_kw(cfg))
    ref.init(*fields)
    t0 = time.perf_counter()
    done = threading.Event()

    def run_oracle():
        ref.step(STEPS)
        done.set()

    th = threading.Thread(target=run_oracle, daemon=True)
    th.start()
    say(f"rb1024 Ra=1e8: oracle {STEPS} steps on {oracle.threads()} threads (background)")
    runs = {}
    for label, storage, rebase in (("f64", "f64", 0), ("f32", "f32", 0), ("bf16s", "bf16s", 0),
                                   ("bf16s+rebase100", "bf16s", 100), ("f16s", "f16s", 0), ("bf16", "bf16", 0)):
        sim = lb.Sim(n, n, scheme="heun", storage=storage, stream=lb.current_stream(), **_kw(cfg))
        sim.set_grid(cfg["xf"], cfg["yf"])
        sim.init(*fields)
        sim.set_rebase(rebase)   # 0: none (the split formats' default is 100)
        sim.step(STEPS)
        r = dict(m=sim.moments(), nu=np.array(sim.nusselt()), d=sim.diagnostics())
        if storage == "f64":
            r["pops"] = sim.populations()
        runs[label] = r
        sim.close()
        say(f"  gpu {label}: done ({time.perf_counter() - t0:.0f} s)")
    while not done.wait(20.0):
        say(f"  oracle still stepping ({time.perf_counter() - t0:.0f} s)")
    th.join()
    say(f"  oracle done ({time.perf_counter() - t0:.0f} s)")
    om = ref.moments()
    od = ref.diagnostics()
    onu = np.array([od["nu_bottom"], od["nu_top"], od["nu_vol"]])
    say(f"  oracle Nu bottom/top/vol = {onu}")
    f, g = runs["f64"]["pops"]
    err = max(np.abs(f - ref.f).max() / np.abs(ref.f).max(), np.abs(g - ref.g).max() / np.abs(ref.g).max())
    say(f"  f64 populations vs oracle: max rel {err:.2e}")
    assert err < 1e-12
    du_ref = om["ux"] ** 2 + om["uy"] ** 2
    for label, r in runs.items():
        m = r["m"]
        nu_err = np.abs(r["nu"] - onu) / np.abs(onu)
        eT = _l2(m["T"], om["T"])
        eu = float(np.sqrt(np.mean((m["ux"] - om["ux"]) ** 2 + (m["uy"] - om["uy"]) ** 2) / np.mean(du_ref)))
        say(f"  {label:16s} Nu rel err {nu_err[0]:.2e} {nu_err[1]:.2e} {nu_err[2]:.2e}  T L2 {eT:.2e}  u L2 {eu:.2e}"
            f"  mass {r['d']['mass'] / od['mass'] - 1:+.2e}")
        assert r["d"]["nonfinite"] == 0.0, label
        if label != "bf16":
            assert nu_err.max() <= 0.01, label
            assert eT <= 1e-3, label
