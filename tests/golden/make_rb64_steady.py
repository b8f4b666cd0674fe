"""Writes rb64_ra1e4_steady.json: the steady convective state of the
Rayleigh-Benard set-up of sec. 5 (tau = tau_g = 1/2, free-fall velocity 0.1,
tanh wall refinement, periodic sides) at Ra = 1e4, Pr = 1 on 64 x 64 cells,
computed by the FP64 oracle with the paper's FV scheme (semi-implicit
collision, Heun advection, QUICK).  Only the oracle and the seeded input
generators are called.

    python tests/golden/make_rb64_steady.py      (about 10 minutes on 8 cores)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

N, RA, STRETCH, SEED, STEPS = 64, 1e4, 1.5, 9, 300000


def main():
    cfg = workloads.rb_config(N, RA, STRETCH, seed_index=SEED)
    kw = dict(thermal=True, wall_y=True, dt=cfg["dt"], tau=cfg["tau"], tau_g=cfg["tau_g"], beta_g=cfg["beta_g"],
              T0=cfg["T0"], T_bottom=cfg["T_bottom"], T_top=cfg["T_top"])
    case = oracle.Case(N, N, scheme="heun", xf=cfg["xf"], yf=cfg["yf"], **kw)
    case.init(cfg["rho"], cfg["ux"], cfg["uy"], cfg["T"])
    nu_last = []
    chunk = STEPS // 10
    for k in range(10):
        case.step(chunk)
        d = case.diagnostics()
        nu_last.append([d["nu_bottom"], d["nu_top"], d["nu_vol"]])
        print(f"{(k + 1) * chunk} steps: Nu {nu_last[-1]}", flush=True)
    m = case.moments()
    d = case.diagnostics()
    out = dict(
        source="FP64 oracle, FV semi-implicit + Heun (eq:semi-heun), QUICK, thermal (sec. 5)",
        config=dict(n=N, Ra=RA, Pr=1.0, stretch=STRETCH, seed_index=SEED, steps=STEPS, dt=cfg["dt"], H=cfg["H"]),
        nu_bottom=d["nu_bottom"], nu_top=d["nu_top"], nu_vol=d["nu_vol"],
        nu_change_last_tenth=[abs(a - b) for a, b in zip(nu_last[-1], nu_last[-2])],
        mass=d["mass"], ekin=d["ekin"], etherm=d["etherm"],
        T_profile=m["T"].mean(axis=1).tolist(),
        speed_rms_profile=np.sqrt((m["ux"] ** 2 + m["uy"] ** 2).mean(axis=1)).tolist(),
    )
    with open(os.path.join(HERE, "rb64_ra1e4_steady.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
