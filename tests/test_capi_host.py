"""C-ABI checks that need no GPU: the library loads, exports every function
that include/lb.h declares, and rejects bad arguments before touching the
device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1505_03271_amd as lb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lb_create", "lb_set_grid", "lb_step", "lb_moments", "lb_nusselt", "lb_init",
                     "lb_destroy", "lb_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = lb.lib()   # the binding's loader (it puts torch's HIP runtime in place first)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"liblb.so lacks {missing}"


def test_grid_helpers_match_the_paper_formula():
    x = lb.grid_tanh(512, 512.0, 2.0)
    assert x[0] == 0.0 and x[-1] == 512.0
    i = np.arange(513)
    ref = 256.0 * (1 + np.tanh((2 * i / 512 - 1) * np.arctanh(np.tanh(2.0))) / np.tanh(2.0))
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-11)
    np.testing.assert_allclose(lb.grid_uniform(8, 2.0), np.arange(9) / 4.0, atol=0)


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=2), "nx and ny"),
    (dict(tau=0.0), "tau"),
    (dict(tau=-1.0), "tau"),
    (dict(dt=0.0), "dt"),
    (dict(scheme="heun", stream_only=True), "STREAM_ONLY"),
    (dict(wall_y="density"), "boundary kind"),
    (dict(wall_x="density", thermal=True, tau_g=0.5), "fixed-density"),
    (dict(wall_x="density", scheme="st"), "fixed-density"),
    (dict(wall_x="density", rho_x0=0.0), "rho_x0"),
    (dict(scheme="st", storage="bf16s"), "moment-split"),
])
def test_create_rejects_bad_parameters(kw, msg):
    args = dict(nx=16, ny=16, scheme="heun", storage="f32", tau=0.5, dt=1.0)
    args.update(kw)
    nx, ny = args.pop("nx"), args.pop("ny")
    with pytest.raises(lb.LBError) as e:
        lb.Sim(nx, ny, **args)
    assert e.value.code == 1 and msg in str(e.value)


def test_bad_storage_and_scheme_codes():
    p = lb.Params(16, 16, 0, 7, 0, 0, 0, 0, 1.0, 0.5, 0.5, 0, 0, 0, 0, 0, 0, 1.0, 0.0, 1.0, 1.0, None)
    h = ctypes.c_void_p()
    assert lb.lib().lb_create(ctypes.byref(p), ctypes.byref(h)) == 1
    assert b"storage" in lb.lib().lb_last_error()
    p.storage, p.scheme = 0, 9
    assert lb.lib().lb_create(ctypes.byref(p), ctypes.byref(h)) == 1
    assert lb.lib().lb_create(None, ctypes.byref(h)) == 1


def test_null_handle_is_rejected():
    assert lb.lib().lb_step(None, 1) == 1
    assert lb.lib().lb_sync(None) == 1
    assert lb.lib().lb_group_step(None, 1) == 1
    assert lb.lib().lb_group_set_chunk(None, 0) == 1
    assert lb.lib().lb_set_st_pairs(None, 1) == 1
    lb.lib().lb_destroy(None)  # no-op
    lb.lib().lb_group_destroy(None)


def test_sinh_and_chebyshev_grids():
    """eq:grids: the sinh grid against the oracle's independent generator and
    its closed-form middle face; the Chebyshev faces (reading with i in place
    of i - 1/2) are symmetric, end at 0 and L, and their cell widths grow
    like sin(i pi / n) away from the walls."""
    import oracle
    x = lb.grid_sinh(64, 64.0, 6.5)
    np.testing.assert_allclose(x, oracle.grid_sinh(64, 64.0, 6.5), rtol=0, atol=1e-12)
    assert x[32] == pytest.approx(32.0, abs=1e-12)
    assert np.all(np.diff(x) > 0) and x[0] == 0.0 and x[-1] == 64.0
    with pytest.raises(lb.LBError):
        lb.grid_sinh(63, 64.0, 6.5)
    c = lb.grid_chebyshev(40, 2.0)
    assert c[0] == 0.0 and c[-1] == 2.0
    np.testing.assert_allclose(c + c[::-1], 2.0, atol=1e-14)
    i = np.arange(40) + 0.5
    np.testing.assert_allclose(np.diff(c), 2.0 * np.sin(i * np.pi / 40) * np.sin(np.pi / 80), rtol=1e-12)



@pytest.mark.parametrize("storage,n,ok", [("bf16s", 9800, True), ("bf16s", 9900, False), ("f64", 5500, False),
                                         ("f32", 7700, True), ("f32", 7800, False)])
def test_state_size_limit(storage, n, ok):
    """A population state must stay below 4 GiB (32-bit buffer offsets):
    thermal 44 B/cell (split), 144 B (F64), 72 B (F32).  Rejected before
    any device allocation; accepted sizes are not created here (no GPU)."""
    per = {"bf16s": 44, "f64": 144, "f32": 72}[storage]
    assert (per * n * n < 2 ** 32) == ok
    if not ok:
        with pytest.raises(lb.LBError) as e:
            lb.Sim(n, n, scheme="heun", storage=storage, thermal=True, tau=0.5, tau_g=0.5, dt=1.0)
        assert e.value.code == 1 and "4 GiB" in str(e.value)


def test_stream_probe_rejects_bad_arguments_before_touching_the_device():
    """lb_stream_probe validates its arguments first: a NULL output or a
    buffer below 16 MiB is LB_EINVAL (no HIP call is made)."""
    L = lb.lib()
    out = (ctypes.c_double * 3)()
    assert L.lb_stream_probe(1 << 20, None, out) == 1
    assert "16 MiB" in L.lb_last_error().decode()
    assert L.lb_stream_probe(64 << 20, None, None) == 1


def test_header_is_plain_c():
    """include/lb.h is a C header (the boundary takes plain pointers and
    sizes): it compiles as C99 and as C++ on its own."""
    import shutil
    import subprocess
    for cc, std, lang in (("gcc", "-std=c99", "c"), ("g++", "-std=c++17", "c++")):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} is not installed")
        r = subprocess.run([cc, "-fsyntax-only", std, "-Wall", "-Werror", "-x", lang,
                            os.path.join(ROOT, "include", "lb.h")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
