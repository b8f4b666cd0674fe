"""Writes rb_onset_rates.json: the growth of the convection rolls just below
and just above the onset of Rayleigh-Benard convection (sec. 5: aspect ratio
2.02, Pr = 1, onset between Ra = 1600 and 1800), computed by the FP64 oracle
with the paper's FV scheme on 48 x 24 cells (uniform cells in y, periodic
sides, isothermal no-slip walls).  The roll energy is the kinetic energy of
the x-varying part of the flow; it is recorded every half diffusion time
H^2 / (2 kappa).  Only the oracle and the seeded input generators are called.

    python tests/golden/make_onset_rates.py      (about 40 s on 8 cores)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

NY, ASPECT, SEED, NOISE, CHECKPOINTS = 24, 2.02, 12, 1e-2, 4


def roll_energy(m):
    du = m["ux"] - m["ux"].mean(axis=1, keepdims=True)
    dv = m["uy"] - m["uy"].mean(axis=1, keepdims=True)
    return 0.5 * float(np.sum(m["rho"] * (du * du + dv * dv)))


def main():
    out = dict(source="FP64 oracle, FV semi-implicit + Heun (eq:semi-heun), QUICK, thermal (sec. 5)",
               config=dict(ny=NY, aspect=ASPECT, Pr=1.0, stretch=1.0, seed_index=SEED, noise=NOISE), runs={})
    for Ra in (1600.0, 1800.0):
        nx = int(round(ASPECT * NY))
        P = workloads.rb_params(Ra, 1.0, nx, NY, aspect=nx / NY, stretch=1.0)
        rho, ux, uy, T = workloads.rb_fields(nx, P["yf"], P["dT"], P["T0"], P["beta_g"], noise=NOISE,
                                             seed_index=SEED)
        case = oracle.Case(nx, NY, scheme="heun", thermal=True, wall_y=True, dt=P["dt"], tau=P["tau"],
                           tau_g=P["tau_g"], beta_g=P["beta_g"], T0=P["T0"], T_bottom=P["T_bottom"],
                           T_top=P["T_top"], xf=P["xf"], yf=P["yf"])
        case.init(rho, ux, uy, T)
        steps = int(0.5 * P["H"] ** 2 / P["kappa"] / P["dt"])
        energy = []
        for _ in range(CHECKPOINTS):
            case.step(steps)
            energy.append(roll_energy(case.moments()))
        print(f"Ra {Ra:.0f}: {steps} steps per checkpoint, roll energy {energy}", flush=True)
        out["runs"][f"{Ra:.0f}"] = dict(nx=nx, steps_per_checkpoint=steps, dt=P["dt"], roll_energy=energy)
    with open(os.path.join(HERE, "rb_onset_rates.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
