"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):

* the oracle (oracle.c, plain C) built with gcc -fsanitize=address,undefined
  and a subset of its pins run against that build;
* the C ABI's host code (capi.cpp: validation, grid helpers, handle and
  group bookkeeping up to the first device call) built with the
  sanitizers on the host side only (-Xarch_host), linked with the kernels
  of the normal build, and driven by tests/capi_host_check.c.

A sanitizer report fails the test (halt on the first error)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, env=None, timeout=600):
    return subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    r = _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
              "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    assert r.returncode == 0, r.stderr
    asan_rt = _run(["gcc", "-print-file-name=libasan.so"]).stdout.strip()
    assert os.path.exists(asan_rt), asan_rt
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan_rt, OMP_NUM_THREADS="2", **SAN_ENV)
    subset = ("brute_force or mass_conservation or momentum_periodic or quick or tanh_grid or relaxation or "
              "fixed_point or conduction or thermal_energy or dirichlet or fixed_density_rest or permutation")
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
              os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", subset], env=env, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out


def test_capi_host_paths_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc")
    objs = [os.path.join(ROOT, "paper_1505_03271_amd", "_build", f + ".o")
            for f in ("fv.hip", "fv3d.hip", "st.hip", "aux.hip", "probe.hip")]
    if hipcc is None or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs hipcc and the kernel objects of __graft_entry__.build()")
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        pytest.skip("needs the ROCm clang for the driver")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    capi_o = str(tmp_path / "capi_san.o")
    r = _run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-x", "hip",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
              "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1505_03271_amd", "csrc"),
              "-Wno-unused-result"] + san + ["-c", os.path.join(ROOT, "paper_1505_03271_amd", "csrc", "capi.cpp"),
                                             "-o", capi_o], timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    lib = str(tmp_path / "liblb_san.so")
    r = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
              "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", lib, capi_o] + objs)
    assert r.returncode == 0, r.stderr[-4000:]
    exe = str(tmp_path / "capi_host_check")
    r = _run([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
              "-shared-libsan", "-I", os.path.join(ROOT, "include"),
              os.path.join(ROOT, "tests", "capi_host_check.c"), "-o", exe, lib, "-Wl,-rpath," + str(tmp_path)])
    assert r.returncode == 0, r.stderr[-4000:]
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so") + \
        glob.glob("/opt/rocm/llvm/lib/clang/*/lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so")
    env = dict(os.environ, **SAN_ENV)
    if rt:
        env["LD_LIBRARY_PATH"] = os.path.dirname(rt[0]) + ":" + env.get("LD_LIBRARY_PATH", "")
    r = _run([exe], env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "host checks passed" in out
