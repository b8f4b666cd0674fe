"""FP64 CPU oracle of the FV-LB and ST-LB steps (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It wraps ``oracle.c`` (plain C, double
precision, OpenMP over rows) through ctypes and shares nothing with the HIP
library in ``paper_1505_03271_amd``.

Schemes: ``"heun"`` (eq:semi-heun, the paper's method), ``"semi"``
(eq:semi), ``"euler"`` (eq:euler) and ``"st"`` (eq:ST).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB: another build of oracle.c (the sanitizer test loads one built
# with -fsanitize=address,undefined)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SCHEMES = {"heun": 0, "semi": 1, "euler": 2, "st": 3}


def build():
    """Compile liboracle.so with gcc (IEEE double, no contraction)."""
    src = os.path.join(HERE, "oracle.c")
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           "-std=c11", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB_PATH)


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("wall_x", ctypes.c_int32), ("wall_y", ctypes.c_int32),
                ("thermal", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("dt", ctypes.c_double), ("tau", ctypes.c_double), ("tau_g", ctypes.c_double),
                ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("beta_g", ctypes.c_double), ("T0", ctypes.c_double),
                ("T_bottom", ctypes.c_double), ("T_top", ctypes.c_double),
                ("rho_lo", ctypes.c_double), ("rho_hi", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        L.ob_abi_version.restype = ctypes.c_int
        L.ob_threads.restype = ctypes.c_int
        L.ob_set_threads.argtypes = [ctypes.c_int]
        L.ob_set_threads.restype = None
        L.ob_set_bracket.argtypes = [ctypes.c_int]
        L.ob_set_bracket.restype = None
        L.ob_grid_uniform.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.ob_grid_tanh.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        L.ob_grid_sinh.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        L.ob_quick_gammas.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp]
        L.ob_init.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L.ob_moments.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L.ob_fv_run.argtypes = [pp, dp, dp, dp, dp, ctypes.c_longlong]
        L.ob_fv_run.restype = ctypes.c_int
        L.ob_st_run.argtypes = [pp, dp, dp, ctypes.c_longlong]
        L.ob_st_run.restype = ctypes.c_int
        L.ob_st_stream_sources.argtypes = [pp, ctypes.POINTER(ctypes.c_int64)]
        L.ob_diagnostics.argtypes = [pp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads():
    return lib().ob_threads()


def set_bracket(alt):
    """Reading of the bracket's force term: False, the literal +dt/2 F (the
    default); True, the Crank-Nicolson physical distribution's
    dt/2 (1 - dt/(2 tau~)) F.  Only for measuring what the reading moves."""
    lib().ob_set_bracket(int(bool(alt)))


def set_threads(n):
    """OpenMP threads of the oracle's loops (timing; results are the same)."""
    lib().ob_set_threads(int(n))


def grid_uniform(n, L):
    out = np.empty(n + 1)
    lib().ob_grid_uniform(n, L, _ptr(out))
    return out


def grid_tanh(n, L, s1):
    """eq:grids, hyperbolic tangent, stretching factor s1 in (0, 1)."""
    out = np.empty(n + 1)
    lib().ob_grid_tanh(n, L, s1, _ptr(out))
    return out


def grid_sinh(n, L, s2):
    out = np.empty(n + 1)
    lib().ob_grid_sinh(n, L, s2, _ptr(out))
    return out


def quick_gammas(faces, periodic):
    faces = np.ascontiguousarray(faces, dtype=np.float64)
    n = len(faces) - 1
    out = np.empty((n + 1, 4))
    lib().ob_quick_gammas(n, _ptr(faces), int(bool(periodic)), _ptr(out))
    return out


class Case:
    """One simulation: parameters, grid and FP64 populations f~, g~ [9][ny][nx]."""

    def __init__(self, nx, ny, scheme="heun", wall_x=False, wall_y=False, thermal=False,
                 dt=1.0, tau=0.5, tau_g=0.5, ax=0.0, ay=0.0, beta_g=0.0, T0=0.0,
                 T_bottom=0.0, T_top=0.0, xf=None, yf=None, rho_lo=1.0, rho_hi=1.0):
        """wall_x, wall_y: False/0 periodic, True/1 no-slip wall, 2 fixed density
        (rho_lo on the low face, rho_hi on the high face of that axis)."""
        self.p = _Params(nx, ny, int(wall_x), int(wall_y), int(thermal), SCHEMES[scheme],
                         float(dt), float(tau), float(tau_g), float(ax), float(ay),
                         float(beta_g), float(T0), float(T_bottom), float(T_top),
                         float(rho_lo), float(rho_hi))
        self.nx, self.ny, self.thermal, self.scheme = nx, ny, thermal, scheme
        self.xf = np.ascontiguousarray(xf if xf is not None else np.arange(nx + 1, dtype=float))
        self.yf = np.ascontiguousarray(yf if yf is not None else np.arange(ny + 1, dtype=float))
        assert len(self.xf) == nx + 1 and len(self.yf) == ny + 1
        self.f = np.zeros((9, ny, nx))
        self.g = np.zeros((9, ny, nx)) if thermal else None

    def init(self, rho, ux, uy, T=None):
        c = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        rho, ux, uy = c(rho), c(ux), c(uy)
        T = c(T) if T is not None else np.zeros_like(rho)
        g = self.g if self.thermal else np.zeros((9, self.ny, self.nx))
        lib().ob_init(ctypes.byref(self.p), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(self.f), _ptr(g))

    def step(self, n=1):
        g = self.g if self.thermal else np.zeros(1)
        if self.scheme == "st":
            rc = lib().ob_st_run(ctypes.byref(self.p), _ptr(self.f), _ptr(g), n)
        else:
            rc = lib().ob_fv_run(ctypes.byref(self.p), _ptr(self.xf), _ptr(self.yf), _ptr(self.f), _ptr(g), n)
        if rc != 0:
            raise RuntimeError(f"oracle step failed ({rc})")

    def moments(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        g = self.g if self.thermal else np.zeros(1)
        lib().ob_moments(ctypes.byref(self.p), _ptr(self.f), _ptr(g), *[_ptr(o) for o in out])
        return dict(rho=out[0], ux=out[1], uy=out[2], T=out[3])

    def diagnostics(self):
        out = np.empty(8)
        g = self.g if self.thermal else np.zeros(1)
        lib().ob_diagnostics(ctypes.byref(self.p), _ptr(self.xf), _ptr(self.yf), _ptr(self.f), _ptr(g), _ptr(out))
        keys = ["mass", "ekin", "etherm", "nu_bottom", "nu_top", "nu_vol", "volume", "nonfinite"]
        return dict(zip(keys, out))

    def stream_sources(self):
        src = np.empty(9 * self.nx * self.ny, dtype=np.int64)
        lib().ob_st_stream_sources(ctypes.byref(self.p), src.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return src

    def brute_params(self):
        p = self.p
        return dict(nx=p.nx, ny=p.ny, wall_x=p.wall_x, wall_y=p.wall_y, thermal=p.thermal, dt=p.dt,
                    tau=p.tau, tau_g=p.tau_g, ax=p.ax, ay=p.ay, beta_g=p.beta_g, T0=p.T0,
                    T_bottom=p.T_bottom, T_top=p.T_top, rho_lo=p.rho_lo, rho_hi=p.rho_hi)


# ---------------------------------------------------------------- 3D -------

class _Params3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("wall", ctypes.c_int32 * 3), ("thermal", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("dt", ctypes.c_double), ("tau", ctypes.c_double), ("tau_g", ctypes.c_double),
                ("a0", ctypes.c_double * 3), ("beta_g", ctypes.c_double), ("T0", ctypes.c_double),
                ("T_bottom", ctypes.c_double), ("T_top", ctypes.c_double)]


def _lib3():
    L = lib()
    if not hasattr(L, "_ob3_ready"):
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params3)
        L.ob3_init.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp]
        L.ob3_moments.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp]
        L.ob3_fv_run.argtypes = [pp, dp, dp, dp, dp, dp, ctypes.c_longlong]
        L.ob3_fv_run.restype = ctypes.c_int
        L.ob3_diagnostics.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L._ob3_ready = True
    return L


class Case3D:
    """One 3D simulation (D3Q19, FV schemes): populations [19][nz][ny][nx];
    z is the vertical axis (gravity, isothermal walls)."""

    def __init__(self, nx, ny, nz, scheme="heun", walls=(False, False, False), thermal=False, dt=1.0,
                 tau=0.5, tau_g=0.5, a=(0.0, 0.0, 0.0), beta_g=0.0, T0=0.0, T_bottom=0.0, T_top=0.0,
                 xf=None, yf=None, zf=None):
        self.p = _Params3(nx, ny, nz, (ctypes.c_int32 * 3)(*[int(w) for w in walls]), int(thermal),
                          SCHEMES[scheme], float(dt), float(tau), float(tau_g),
                          (ctypes.c_double * 3)(*[float(v) for v in a]), float(beta_g), float(T0),
                          float(T_bottom), float(T_top))
        self.n = (nx, ny, nz)
        self.thermal = thermal
        f = lambda v, n: np.ascontiguousarray(v if v is not None else np.arange(n + 1, dtype=float), dtype=float)
        self.xf, self.yf, self.zf = f(xf, nx), f(yf, ny), f(zf, nz)
        self.f = np.zeros((19, nz, ny, nx))
        self.g = np.zeros((19, nz, ny, nx)) if thermal else None

    def init(self, rho, ux, uy, uz, T=None):
        c = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        rho, ux, uy, uz = c(rho), c(ux), c(uy), c(uz)
        T = c(T) if T is not None else np.zeros_like(rho)
        g = self.g if self.thermal else np.zeros_like(self.f)
        _lib3().ob3_init(ctypes.byref(self.p), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz), _ptr(T), _ptr(self.f),
                         _ptr(g))

    def step(self, n=1):
        g = self.g if self.thermal else np.zeros(1)
        rc = _lib3().ob3_fv_run(ctypes.byref(self.p), _ptr(self.xf), _ptr(self.yf), _ptr(self.zf), _ptr(self.f),
                                _ptr(g), n)
        if rc != 0:
            raise RuntimeError(f"oracle 3D step failed ({rc})")

    def moments(self):
        shape = self.f.shape[1:]
        out = {k: np.empty(shape) for k in ("rho", "ux", "uy", "uz", "T")}
        g = self.g if self.thermal else np.zeros_like(self.f)
        _lib3().ob3_moments(ctypes.byref(self.p), _ptr(self.f), _ptr(g), _ptr(out["rho"]), _ptr(out["ux"]),
                            _ptr(out["uy"]), _ptr(out["uz"]), _ptr(out["T"]))
        return out

    def diagnostics(self):
        out = np.empty(8)
        g = self.g if self.thermal else np.zeros_like(self.f)
        _lib3().ob3_diagnostics(ctypes.byref(self.p), _ptr(self.xf), _ptr(self.yf), _ptr(self.zf), _ptr(self.f),
                                _ptr(g), _ptr(out))
        keys = ("mass", "ekin", "etherm", "nu_bottom", "nu_top", "nu_vol", "volume", "nonfinite")
        return dict(zip(keys, out))

    def brute_params(self):
        p = self.p
        return dict(n=tuple(self.n), wall=tuple(p.wall), thermal=p.thermal, dt=p.dt, tau=p.tau, tau_g=p.tau_g,
                    a=tuple(p.a0), beta_g=p.beta_g, T0=p.T0, T_bottom=p.T_bottom, T_top=p.T_top)
