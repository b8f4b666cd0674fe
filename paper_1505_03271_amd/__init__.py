"""Python binding of liblb (include/lb.h): argument marshalling only.

Every step of the FV-LB / ST-LB path runs in the HIP kernels of liblb.so;
this module converts NumPy arrays and torch streams into the C ABI's plain
pointers.  It raises if liblb.so has not been built: there is no fallback.

    import paper_1505_03271_amd as lb
    sim = lb.Sim(nx, ny, scheme="heun", storage="bf16", thermal=True, ...)
    sim.set_grid(x_faces, y_faces)
    sim.init(rho, ux, uy, T)
    sim.step(1000)
    nu_bottom, nu_top, nu_vol = sim.nusselt()
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# LB_LIB: another build of the library (the sanitizer and tuning builds)
LIB_PATH = os.environ.get("LB_LIB") or os.path.join(PKG, "liblb.so")

SCHEMES = {"heun": 0, "semi": 1, "euler": 2, "st": 3}
STORAGE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "bf16s": 4, "f16s": 5}
STORAGE_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}


def cell_bytes(storage, thermal=True):
    """Bytes of one cell of one population state in `storage`."""
    if storage in ("bf16s", "f16s"):   # float moments + 16-bit residuals
        return 44 if thermal else 24
    return (18 if thermal else 9) * STORAGE_BYTES[storage]


FLAG_STREAM_ONLY = 1
# boundary kinds per axis: periodic, no-slip wall, fixed density (x only)
BOUNDARY = {False: 0, True: 1, 0: 0, 1: 1, 2: 2, "periodic": 0, "wall": 1, "density": 2}
STATUS = {0: "LB_OK", 1: "LB_EINVAL", 2: "LB_ENOMEM", 3: "LB_EDEVICE", 4: "LB_ESTATE", 5: "LB_EUNSTABLE"}


class LBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("thermal", ctypes.c_int32), ("bc_x", ctypes.c_int32),
                ("bc_y", ctypes.c_int32), ("flags", ctypes.c_int32), ("dt", ctypes.c_double),
                ("tau", ctypes.c_double), ("tau_g", ctypes.c_double), ("ax", ctypes.c_double),
                ("ay", ctypes.c_double), ("beta_g", ctypes.c_double), ("T0", ctypes.c_double),
                ("T_bottom", ctypes.c_double), ("T_top", ctypes.c_double), ("rho_ref", ctypes.c_double),
                ("T_ref", ctypes.c_double), ("rho_x0", ctypes.c_double), ("rho_x1", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class Params3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("storage", ctypes.c_int32), ("thermal", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3), ("dt", ctypes.c_double), ("tau", ctypes.c_double),
                ("tau_g", ctypes.c_double), ("a", ctypes.c_double * 3), ("beta_g", ctypes.c_double),
                ("T0", ctypes.c_double), ("T_bottom", ctypes.c_double), ("T_top", ctypes.c_double),
                ("rho_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("stream", ctypes.c_void_p)]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load liblb.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        # torch ships its own HIP runtime under the same soname as the system
        # one liblb links against; whichever is loaded first serves the whole
        # process.  Load torch's first so that torch and liblb share it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        h = ctypes.c_void_p
        sig = {
            "lb_create": ([ctypes.POINTER(Params), ctypes.POINTER(h)], ctypes.c_int),
            "lb_destroy": ([h], None),
            "lb_set_grid": ([h, _DP, ctypes.c_int64, _DP, ctypes.c_int64], ctypes.c_int),
            "lb_grid_uniform": ([ctypes.c_int64, ctypes.c_double, _DP], ctypes.c_int),
            "lb_grid_tanh": ([ctypes.c_int64, ctypes.c_double, ctypes.c_double, _DP], ctypes.c_int),
            "lb_grid_sinh": ([ctypes.c_int64, ctypes.c_double, ctypes.c_double, _DP], ctypes.c_int),
            "lb_grid_chebyshev": ([ctypes.c_int64, ctypes.c_double, _DP], ctypes.c_int),
            "lb_profiles": ([h, _DP, ctypes.c_int64], ctypes.c_int),
            "lb_init": ([h, _DP, _DP, _DP, _DP], ctypes.c_int),
            "lb_step": ([h, ctypes.c_int64], ctypes.c_int),
            "lb_sync": ([h], ctypes.c_int),
            "lb_moments": ([h, _DP, _DP, _DP, _DP], ctypes.c_int),
            "lb_nusselt": ([h, _DP, _DP, _DP], ctypes.c_int),
            "lb_diagnostics": ([h, _DP], ctypes.c_int),
            "lb_diagnostics_noalloc": ([h, ctypes.c_void_p], ctypes.c_int),
            "lb_get_populations": ([h, _DP, _DP], ctypes.c_int),
            "lb_set_populations": ([h, _DP, _DP], ctypes.c_int),
            "lb_state_bytes": ([h], ctypes.c_size_t),
            "lb_get_state": ([h, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
            "lb_set_state": ([h, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
            "lb_set_timing": ([h, ctypes.c_int], ctypes.c_int),
            "lb_kernel_times": ([h, ctypes.POINTER(ctypes.c_int64), _DP], ctypes.c_int),
            "lb_set_fv_chunk": ([h, ctypes.c_int], ctypes.c_int),
            "lb_set_fv_lanes": ([h, ctypes.c_int], ctypes.c_int),
            "lb_set_fv_fused": ([h, ctypes.c_int], ctypes.c_int),
            "lb_get_fv_fused": ([h, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
            "lb_set_st_pairs": ([h, ctypes.c_int], ctypes.c_int),
            "lb_rebase": ([h], ctypes.c_int),
            "lb_set_rebase": ([h, ctypes.c_int64], ctypes.c_int),
            "lb_device_bytes": ([h], ctypes.c_size_t),
            "lb_last_error": ([], ctypes.c_char_p),
            "lb_stream_probe": ([ctypes.c_size_t, ctypes.c_void_p, _DP], ctypes.c_int),
            "lb_group_create": ([ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(h)], ctypes.c_int),
            "lb_group_destroy": ([h], None),
            "lb_group_add": ([h, h, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "lb_group_remove": ([h, ctypes.c_int32], ctypes.c_int),
            "lb_group_set_chunk": ([h, ctypes.c_int32], ctypes.c_int),
            "lb_group_step": ([h, ctypes.c_int64], ctypes.c_int),
            "lb_group_sync": ([h], ctypes.c_int),
            "lb_group_remaining": ([h, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
            "lb3_create": ([ctypes.POINTER(Params3), ctypes.POINTER(h)], ctypes.c_int),
            "lb3_destroy": ([h], None),
            "lb3_set_grid": ([h, _DP, ctypes.c_int64, _DP, ctypes.c_int64, _DP, ctypes.c_int64], ctypes.c_int),
            "lb3_init": ([h, _DP, _DP, _DP, _DP, _DP], ctypes.c_int),
            "lb3_step": ([h, ctypes.c_int64], ctypes.c_int),
            "lb3_sync": ([h], ctypes.c_int),
            "lb3_moments": ([h, _DP, _DP, _DP, _DP, _DP], ctypes.c_int),
            "lb3_get_populations": ([h, _DP, _DP], ctypes.c_int),
            "lb3_diagnostics": ([h, _DP], ctypes.c_int),
            "lb3_set_update": ([h, ctypes.c_int], ctypes.c_int),
            "lb3_set_timing": ([h, ctypes.c_int], ctypes.c_int),
            "lb3_kernel_times": ([h, ctypes.POINTER(ctypes.c_int64), _DP], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise LBError(rc, lib().lb_last_error().decode())


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, "expected C-contiguous float64"
    return a.ctypes.data_as(_DP)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = np.ascontiguousarray(np.broadcast_to(a, shape))
    return a


def grid_uniform(n, L):
    out = np.empty(n + 1)
    _check(lib().lb_grid_uniform(n, L, _dptr(out)))
    return out


def grid_tanh(n, L, stretch):
    out = np.empty(n + 1)
    _check(lib().lb_grid_tanh(n, L, stretch, _dptr(out)))
    return out


def grid_sinh(n, L, s2):
    out = np.empty(n + 1)
    _check(lib().lb_grid_sinh(n, L, s2, _dptr(out)))
    return out


def grid_chebyshev(n, L):
    out = np.empty(n + 1)
    _check(lib().lb_grid_chebyshev(n, L, _dptr(out)))
    return out


def stream_probe(bytes_per_buffer=512 << 20, stream=None):
    """lb_stream_probe: best streaming bandwidth of the device in GB/s, as a
    dict copy_1r1w / stream_2r1w / read_2r (a reference ceiling for the stage
    kernels, not part of the method)."""
    out = np.zeros(3)
    _check(lib().lb_stream_probe(int(bytes_per_buffer), stream if stream is not None else current_stream(),
                                 _dptr(out)))
    return dict(copy_1r1w=float(out[0]), stream_2r1w=float(out[1]), read_2r=float(out[2]))


def current_stream():
    """hipStream_t of torch's current stream on the current device."""
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Sim:
    """One simulation handle (lb_create ... lb_destroy)."""

    def __init__(self, nx, ny, scheme="heun", storage="f64", thermal=False, wall_x=False, wall_y=False,
                 dt=1.0, tau=0.5, tau_g=0.5, ax=0.0, ay=0.0, beta_g=0.0, T0=0.0, T_bottom=0.0, T_top=0.0,
                 rho_ref=1.0, T_ref=0.0, stream=None, stream_only=False, rho_x0=1.0, rho_x1=1.0):
        """wall_x, wall_y: False/"periodic", True/"wall", or (x only) "density"
        with the face densities rho_x0, rho_x1."""
        self.nx, self.ny, self.thermal = nx, ny, bool(thermal)
        self.scheme, self.storage = scheme, storage
        self.p = Params(nx, ny, SCHEMES[scheme], STORAGE[storage], int(bool(thermal)), BOUNDARY[wall_x],
                        BOUNDARY[wall_y], FLAG_STREAM_ONLY if stream_only else 0, float(dt), float(tau),
                        float(tau_g), float(ax), float(ay), float(beta_g), float(T0), float(T_bottom),
                        float(T_top), float(rho_ref), float(T_ref), float(rho_x0), float(rho_x1),
                        stream.value if isinstance(stream, ctypes.c_void_p) else stream)
        self.h = ctypes.c_void_p()
        _check(lib().lb_create(ctypes.byref(self.p), ctypes.byref(self.h)))

    def close(self):
        if self.h:
            lib().lb_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_grid(self, x_faces, y_faces):
        x, y = _f64(x_faces), _f64(y_faces)
        _check(lib().lb_set_grid(self.h, _dptr(x), len(x), _dptr(y), len(y)))

    def init(self, rho, ux, uy, T=None):
        shp = (self.ny, self.nx)
        r, u, v = _f64(rho, shp), _f64(ux, shp), _f64(uy, shp)
        t = _f64(T, shp) if T is not None else None
        _check(lib().lb_init(self.h, _dptr(r), _dptr(u), _dptr(v), _dptr(t)))

    def step(self, n=1):
        _check(lib().lb_step(self.h, int(n)))

    def sync(self):
        _check(lib().lb_sync(self.h))

    def moments(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        _check(lib().lb_moments(self.h, *[_dptr(o) for o in out]))
        return dict(rho=out[0], ux=out[1], uy=out[2], T=out[3])

    def profiles(self):
        """Per-row x averages (lb_profiles): dict of [ny] arrays T_mean,
        T_rms, ux_rms, uy_rms, uyT, Nu."""
        out = np.empty(6 * self.ny)
        _check(lib().lb_profiles(self.h, _dptr(out), out.size))
        out = out.reshape(6, self.ny)
        return dict(T_mean=out[0], T_rms=out[1], ux_rms=out[2], uy_rms=out[3], uyT=out[4], Nu=out[5])

    def nusselt(self):
        b, t, v = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().lb_nusselt(self.h, ctypes.byref(b), ctypes.byref(t), ctypes.byref(v)))
        return b.value, t.value, v.value

    def diagnostics_noalloc(self, out_device_ptr):
        """lb_diagnostics_noalloc: enqueue the eight values into a device
        array of 8 doubles at out_device_ptr (an integer address); returns at
        once."""
        _check(lib().lb_diagnostics_noalloc(self.h, ctypes.c_void_p(int(out_device_ptr))))

    def diagnostics(self):
        out = np.empty(8)
        _check(lib().lb_diagnostics(self.h, _dptr(out)))
        keys = ["mass", "ekin", "etherm", "nu_bottom", "nu_top", "nu_vol", "volume", "nonfinite"]
        return dict(zip(keys, out))

    def populations(self):
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((9, self.ny, self.nx)) if self.thermal else None
        _check(lib().lb_get_populations(self.h, _dptr(f), _dptr(g)))
        return f, g

    def set_populations(self, f, g=None):
        shp = (9, self.ny, self.nx)
        f = _f64(f, shp)
        g = _f64(g, shp) if self.thermal else None
        _check(lib().lb_set_populations(self.h, _dptr(f), _dptr(g)))

    def state_bytes(self):
        return lib().lb_state_bytes(self.h)

    def get_state(self):
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        _check(lib().lb_get_state(self.h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))
        return buf

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf).view(np.uint8).reshape(-1)
        _check(lib().lb_set_state(self.h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))

    def set_timing(self, on=True):
        _check(lib().lb_set_timing(self.h, int(bool(on))))

    def kernel_times(self):
        n = (ctypes.c_int64 * 4)()
        ms = (ctypes.c_double * 4)()
        _check(lib().lb_kernel_times(self.h, n, ms))
        names = ["fv_first_pass", "fv_corrector", "st", "fv_fused"]
        return {names[k]: (int(n[k]), float(ms[k])) for k in range(4)}

    def set_fv_fused(self, on):
        """on: 1 (True) fused steps wherever they apply, 0 (False) never,
        -1 (None) where they pay (the default)."""
        _check(lib().lb_set_fv_fused(self.h, -1 if on is None else int(on)))

    def fv_fused(self):
        """The setting: 1, 0 or -1 (automatic)."""
        on = ctypes.c_int()
        _check(lib().lb_get_fv_fused(self.h, ctypes.byref(on)))
        return on.value

    def rebase(self):
        _check(lib().lb_rebase(self.h))

    def set_rebase(self, every):
        _check(lib().lb_set_rebase(self.h, int(every)))

    def set_fv_lanes(self, lanes):
        _check(lib().lb_set_fv_lanes(self.h, int(lanes)))

    def set_st_pairs(self, on):
        _check(lib().lb_set_st_pairs(self.h, int(bool(on))))

    def set_fv_chunk(self, rows):
        _check(lib().lb_set_fv_chunk(self.h, int(rows)))

    def device_bytes(self):
        return lib().lb_device_bytes(self.h)


class Group:
    """Serving group (lb_group_*): members advance together in shared
    launches, each stopping exactly at its own step count."""

    def __init__(self, max_sims, stream=None):
        self.max_sims = int(max_sims)
        self.h = ctypes.c_void_p()
        st = stream.value if isinstance(stream, ctypes.c_void_p) else stream
        _check(lib().lb_group_create(self.max_sims, st, ctypes.byref(self.h)))
        self.members = {}

    def close(self):
        if self.h:
            lib().lb_group_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, sim, steps):
        slot = ctypes.c_int32()
        _check(lib().lb_group_add(self.h, sim.h, int(steps), ctypes.byref(slot)))
        self.members[slot.value] = sim
        return slot.value

    def remove(self, slot):
        _check(lib().lb_group_remove(self.h, int(slot)))
        self.members.pop(slot, None)

    def set_chunk(self, rows):
        """Rows per work item (0: chosen at each membership change)."""
        _check(lib().lb_group_set_chunk(self.h, int(rows)))

    def step(self, n):
        _check(lib().lb_group_step(self.h, int(n)))

    def sync(self):
        _check(lib().lb_group_sync(self.h))

    def remaining(self):
        out = (ctypes.c_int64 * self.max_sims)()
        _check(lib().lb_group_remaining(self.h, out))
        return list(out)


class Sim3:
    """A 3D simulation (D3Q19, FV schemes; lb3_create ... lb3_destroy).  z is
    the vertical axis: gravity and the isothermal walls are along z."""

    def __init__(self, nx, ny, nz, scheme="heun", storage="f64", thermal=False, walls=(False, False, False),
                 dt=1.0, tau=0.5, tau_g=0.5, a=(0.0, 0.0, 0.0), beta_g=0.0, T0=0.0, T_bottom=0.0, T_top=0.0,
                 rho_ref=1.0, T_ref=0.0, stream=None):
        self.n = (nx, ny, nz)
        self.thermal = bool(thermal)
        self.p = Params3(nx, ny, nz, SCHEMES[scheme], STORAGE[storage], int(bool(thermal)),
                         (ctypes.c_int32 * 3)(*[BOUNDARY[w] for w in walls]), float(dt), float(tau), float(tau_g),
                         (ctypes.c_double * 3)(*[float(v) for v in a]), float(beta_g), float(T0), float(T_bottom),
                         float(T_top), float(rho_ref), float(T_ref),
                         stream.value if isinstance(stream, ctypes.c_void_p) else stream)
        self.h = ctypes.c_void_p()
        _check(lib().lb3_create(ctypes.byref(self.p), ctypes.byref(self.h)))

    def close(self):
        if self.h:
            lib().lb3_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_grid(self, xf, yf, zf):
        x, y, z = _f64(xf), _f64(yf), _f64(zf)
        _check(lib().lb3_set_grid(self.h, _dptr(x), x.size, _dptr(y), y.size, _dptr(z), z.size))

    def init(self, rho, ux, uy, uz, T=None):
        shape = self.n[::-1]
        arrs = [_f64(v, shape) for v in (rho, ux, uy, uz)]
        t = _f64(T, shape) if T is not None else None
        _check(lib().lb3_init(self.h, *[_dptr(v) for v in arrs], _dptr(t) if t is not None else None))

    def step(self, n=1):
        _check(lib().lb3_step(self.h, int(n)))

    def sync(self):
        _check(lib().lb3_sync(self.h))

    def moments(self):
        shape = self.n[::-1]
        out = {k: np.empty(shape) for k in ("rho", "ux", "uy", "uz", "T")}
        _check(lib().lb3_moments(self.h, *[_dptr(out[k]) for k in ("rho", "ux", "uy", "uz", "T")]))
        return out

    def populations(self):
        shape = (19,) + self.n[::-1]
        f = np.empty(shape)
        g = np.empty(shape) if self.thermal else None
        _check(lib().lb3_get_populations(self.h, _dptr(f), _dptr(g) if g is not None else None))
        return f, g

    def diagnostics(self):
        out = np.empty(8)
        _check(lib().lb3_diagnostics(self.h, _dptr(out)))
        keys = ("mass", "ekin", "etherm", "nu_bottom", "nu_top", "nu_vol", "volume", "nonfinite")
        return dict(zip(keys, out.tolist()))

    def set_update(self, kind):
        """Flux + update kernel: "tiled" (LDS tiles, default) or "gather" (one
        thread per cell); results are bit-identical."""
        _check(lib().lb3_set_update(self.h, {"tiled": 0, "gather": 1}[kind]))

    def set_timing(self, on=True):
        _check(lib().lb3_set_timing(self.h, int(bool(on))))

    def kernel_times(self):
        n = (ctypes.c_int64 * 2)()
        ms = (ctypes.c_double * 2)()
        _check(lib().lb3_kernel_times(self.h, n, ms))
        return {"fv_first_pass": (n[0], ms[0]), "fv_corrector": (n[1], ms[1])}
