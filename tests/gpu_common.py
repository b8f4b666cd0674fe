"""Helpers shared by the GPU tests: run the same seeded case through liblb
(HIP) and through the FP64 oracle."""
import numpy as np

import oracle
import paper_1505_03271_amd as lb

# storage unit roundoff (half an ulp relative to the stored magnitude)
UNIT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -9, "f16": 2.0 ** -11, "bf16s": 2.0 ** -9,
        "f16s": 2.0 ** -11}

_OKEYS = ("thermal", "wall_x", "wall_y", "dt", "tau", "tau_g", "ax", "ay", "beta_g", "T0", "T_bottom", "T_top")


def make_pair(nx, ny, scheme, storage, xf, yf, fields, chunk=None, **kw):
    """(gpu Sim, oracle Case) initialised from the same fields."""
    import torch
    sim = lb.Sim(nx, ny, scheme=scheme, storage=storage, stream=lb.current_stream(), **kw)
    sim.set_grid(xf, yf)
    if chunk:
        sim.set_fv_chunk(chunk)
    sim.init(*fields)
    okw = {k: v for k, v in kw.items() if k in _OKEYS}
    if kw.get("wall_x") == "density":
        okw.update(wall_x=2, rho_lo=kw.get("rho_x0", 1.0), rho_hi=kw.get("rho_x1", 1.0))
    ref = oracle.Case(nx, ny, scheme=scheme, xf=xf, yf=yf, **okw)
    ref.init(*fields)
    torch.cuda.synchronize()
    return sim, ref


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def offsets(p, ref_value):
    """population minus w_a * ref (what the narrow formats store)."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    return p - w * ref_value


def random_fields(nx, ny, seed, thermal=True, amp=0.03):
    r = np.random.default_rng(seed)
    rho = 1.0 + 0.01 * r.standard_normal((ny, nx))
    ux = amp * r.standard_normal((ny, nx))
    uy = amp * r.standard_normal((ny, nx))
    T = 0.3 * r.uniform(-1, 1, (ny, nx)) if thermal else None
    return (rho, ux, uy, T) if thermal else (rho, ux, uy)


def residual_scale(f, g, dt, ax, ay, beta_g, T0):
    """max |f~ - (f_eq - dt/2 F)| and |g - g_eq| of an FP64 state: the size
    of what moment-split storage rounds to 16 bits."""
    c = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    cx, cy = c[:, 0, None, None], c[:, 1, None, None]
    rho = f.sum(0)
    T = g.sum(0) if g is not None else 0.0
    Ay = ay + beta_g * (T - T0)
    ux = (cx * f).sum(0) / rho + 0.5 * dt * ax
    uy = (cy * f).sum(0) / rho + 0.5 * dt * Ay
    cu = cx * ux + cy * uy
    ca = cx * ax + cy * Ay
    poly = 1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy)
    frc = 3 * (ca - (ux * ax + uy * Ay)) + 9 * cu * ca
    r = np.abs(f - w * rho * (poly - 0.5 * dt * frc)).max()
    if g is not None:
        r = max(r, np.abs(g - w * T * poly).max())
    return r


def storage_bound(storage, ref, steps, kw):
    """max abs population error allowed after `steps` FV steps in a 16-bit
    storage format against the oracle state `ref`: a few half-ulps per step
    of what the format rounds (the largest stored offset, or for split
    formats the largest residual from the forced equilibrium) plus FP32
    arithmetic on values of size |f| <= 1."""
    u = UNIT[storage]
    if storage in ("bf16s", "f16s"):
        scale = residual_scale(ref.f, ref.g, kw["dt"], kw.get("ax", 0.0), kw.get("ay", 0.0), kw.get("beta_g", 0.0),
                               kw.get("T0", 0.0))
    else:
        scale = max(np.abs(offsets(ref.f, 1.0)).max(), np.abs(ref.g).max() if ref.g is not None else 0.0)
    return steps * (8 * u * scale + 64 * 2.0 ** -24)
