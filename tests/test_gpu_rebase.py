"""The per-row references of narrow thermal storage (T_ref and, for the
moment-split formats, the heat-flux reference q) and their renewal by
lb_rebase, through the C ABI."""
import sys

import numpy as np
import pytest

import paper_1505_03271_amd as lb  # noqa: F401  (the binding under test)
import workloads
from gpu_common import UNIT, make_pair, random_fields

pytestmark = pytest.mark.gpu

KW = dict(thermal=True, wall_y=True, dt=0.5, tau=0.3, tau_g=0.25, ax=1e-5, ay=-2e-5, beta_g=1e-3, T0=0.05,
          T_bottom=0.5, T_top=-0.5)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(storage, nx=160, ny=48, chunk=None, seed=21):
    xf, yf = workloads.faces_uniform(nx, 3.0 * nx), workloads.faces_tanh(ny, 3.0 * ny, 2.0)
    return make_pair(nx, ny, "heun", storage, xf, yf, random_fields(nx, ny, seed), chunk=chunk, **KW)


@pytest.mark.parametrize("storage", ["bf16s", "f16s", "bf16", "f32"])
def test_rebase_changes_the_populations_by_one_rounding(storage):
    """A rebase only re-expresses the stored words: f is untouched and g
    moves by at most one rounding of its re-encoded words (16-bit residuals
    or offsets, bounded by the unit roundoff times |g|), plus FP32 rounding
    of the temperature moment."""
    say(f"rebase {storage}")
    sim, _ = _case(storage)
    sim.step(30)
    f0, g0 = sim.populations()
    sim.rebase()
    f1, g1 = sim.populations()
    u = UNIT[storage]
    say(f"  |df| {np.abs(f1 - f0).max():.2e}  |dg| {np.abs(g1 - g0).max():.2e}  u*|g| {u * np.abs(g0).max():.2e}")
    assert np.abs(f1 - f0).max() <= 4 * 2.0 ** -24
    assert np.abs(g1 - g0).max() <= u * np.abs(g0).max() + 8 * 2.0 ** -24


@pytest.mark.parametrize("storage", ["bf16s", "f16s"])
def test_split_parity_with_a_rebase_every_other_step(storage):
    """References renewed every second step add one rounding per rebase: the
    error against the FP64 oracle stays within a small multiple of the error
    of the same run without rebase."""
    say(f"split parity with rebase {storage}")
    sim, ref = _case(storage, chunk=16)
    plain, _ = _case(storage, chunk=16)
    sim.set_rebase(2)
    for k in range(3):
        sim.step(2)
        plain.step(2)
        ref.step(2)
        f, g = sim.populations()
        fp, gp = plain.populations()
        ef, eg = np.abs(f - ref.f).max(), np.abs(g - ref.g).max()
        efp, egp = np.abs(fp - ref.f).max(), np.abs(gp - ref.g).max()
        say(f"  step {2 * (k + 1)}: err f {ef:.2e} g {eg:.2e}  (no rebase: {efp:.2e} {egp:.2e})")
        assert ef <= 4 * efp + 1e-6 and eg <= 4 * egp + 1e-6


@pytest.mark.parametrize("storage", ["bf16s", "bf16"])
def test_checkpoint_carries_the_references(storage):
    """A state saved after rebases have renewed the references, restored into
    a fresh handle (whose own references are those of lb_init), steps on
    bit-identically: the checkpoint carries the references."""
    say(f"checkpoint with references {storage}")
    sim, _ = _case(storage)
    sim.set_rebase(3)
    sim.step(10)
    sim.set_rebase(0)
    saved = sim.get_state()
    sim.step(7)
    a = sim.get_state()
    other, _ = _case(storage)
    other.set_state(saved)
    other.step(7)
    assert np.array_equal(other.get_state(), a)
