"""Python binding of libswe_hip.so (argument marshalling only).

Every step of the CSPH-TVD path runs in the library's HIP kernels on the GPU;
this module converts NumPy arrays to the C ABI of ``include/swe.h`` and back.
PyTorch is used, when present, only to hand the library the caller's current
HIP stream.  There is no CPU fallback: if the library is missing, importing
the binding raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswe_hip.so")

SWE_OK, SWE_EINVAL, SWE_ENOMEM, SWE_EHIP, SWE_ENONFINITE, SWE_EDTCOLLAPSE = 0, -1, -2, -3, -4, -5
_ERRNAME = {-1: "SWE_EINVAL", -2: "SWE_ENOMEM", -3: "SWE_EHIP", -4: "SWE_ENONFINITE",
            -5: "SWE_EDTCOLLAPSE"}

_dp = ctypes.POINTER(ctypes.c_double)


class SweParams(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int), ("g", ctypes.c_double), ("cfl", ctypes.c_double),
        ("eps", ctypes.c_double), ("dt_max", ctypes.c_double), ("dt_min", ctypes.c_double),
        ("nu", ctypes.c_double), ("f_coriolis", ctypes.c_double),
        ("wind_x", ctypes.c_double), ("wind_y", ctypes.c_double),
        ("wind_kappa", ctypes.c_double), ("h_wind", ctypes.c_double),
        ("limiter", ctypes.c_int), ("skip_dry", ctypes.c_int),
        ("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int),
        ("inlet_i0", ctypes.c_int), ("inlet_j0", ctypes.c_int),
        ("inlet_ni", ctypes.c_int), ("inlet_nj", ctypes.c_int),
        ("q_base", ctypes.c_double), ("q_peak", ctypes.c_double),
        ("t_peak", ctypes.c_double), ("sigma_t", ctypes.c_double),
        ("solid", ctypes.POINTER(ctypes.c_uint8)), ("H0", _dp), ("Qx0", _dp), ("Qy0", _dp),
        ("stream", ctypes.c_void_p), ("sph_displaced", ctypes.c_int), ("periodic", ctypes.c_int),
    ]


class SwePatch(ctypes.Structure):
    """Mirror of swe_patch in swe.h."""
    _fields_ = [("ci0", ctypes.c_int), ("cj0", ctypes.c_int), ("cw", ctypes.c_int), ("ch", ctypes.c_int),
                ("b", _dp), ("n_M", _dp), ("H0", _dp), ("Qx0", _dp), ("Qy0", _dp)]


NEST_FRAME = 5   # SWE_NEST_FRAME


# Every function declared in include/swe.h, with its ctypes signature.
EXPORTS = {
    "swe_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp,
                                     ctypes.POINTER(SweParams)]),
    "swe_step": (ctypes.c_int, [ctypes.c_void_p]),
    "swe_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long]),
    "swe_mass": (ctypes.c_double, [ctypes.c_void_p]),
    "swe_destroy": (None, [ctypes.c_void_p]),
    "swe_get_state": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp]),
    "swe_set_state": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp]),
    "swe_set_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "swe_time": (ctypes.c_double, [ctypes.c_void_p]),
    "swe_last_dt": (ctypes.c_double, [ctypes.c_void_p]),
    "swe_next_dt": (ctypes.c_double, [ctypes.c_void_p]),
    "swe_ledger": (ctypes.c_double, [ctypes.c_void_p]),
    "swe_inflow": (ctypes.c_double, [ctypes.c_void_p]),
    "swe_steps": (ctypes.c_long, [ctypes.c_void_p]),
    "swe_launch_grid": (ctypes.c_int, [ctypes.c_void_p]),
    "swe_set_launch_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "swe_enqueue": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long]),
    "swe_step_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
                         + [ctypes.c_void_p] * 8 + [ctypes.c_double, ctypes.c_void_p]),
    "swe_set_source_field": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "swe_field_volume": (ctypes.c_double, [ctypes.c_void_p]),
    "swe_work": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong),
                                ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "swe_active_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "swe_run_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long, _dp]),
    "swe_batch_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), _dp, ctypes.POINTER(_dp),
                                           ctypes.POINTER(_dp), ctypes.POINTER(SweParams)]),
    "swe_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, ctypes.POINTER(SweParams),
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), _dp]),
    "swe_batch_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                          _dp, ctypes.POINTER(_dp), ctypes.POINTER(_dp), ctypes.POINTER(SweParams),
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int), _dp]),
    "swe_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long]),
    "swe_batch_run_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long, _dp]),
    "swe_batch_query": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_long)]),
    "swe_batch_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]),
    "swe_batch_work": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)]),
    "swe_batch_destroy": (None, [ctypes.c_void_p]),
    "swe_nest_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp,
                                          ctypes.POINTER(SweParams), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p]),
    "swe_nest_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long]),
    "swe_nest_hold_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "swe_nest_run_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long, _dp]),
    "swe_nest_query": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_long),
                                      _dp, _dp]),
    "swe_nest_get_coarse": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp]),
    "swe_nest_get_patch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]),
    "swe_nest_destroy": (None, [ctypes.c_void_p]),
    "swe_nest_work": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.POINTER(ctypes.c_longlong)]),
    "swe_set_correction": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "swe_set_correction_depth": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "swe_hold_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "swe_enable_line_taps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "swe_zero_line_taps": (ctypes.c_int, [ctypes.c_void_p]),
    "swe_get_line_taps": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp]),
    "swe_restrict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "swe_lc_nparams": (ctypes.c_int, []),
    "swe_lc_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_void_p]),
    "swe_lc_destroy": (None, [ctypes.c_void_p]),
    "swe_lc_set_params": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "swe_lc_get_params": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "swe_lc_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp]),
    "swe_lc_infer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp]),
    "swe_lc_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _dp]),
    "swe_lc_get_grads": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "swe_lc_get_layer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "swe_lc_attach": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "swe_lc_data": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "swe_lc_set_out_scale": (ctypes.c_int, [ctypes.c_void_p, _dp]),
    "swe_lc_data_count": (ctypes.c_int, [ctypes.c_void_p]),
    "swe_lc_collect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                      _dp]),
    "swe_lc_get_data": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
                                       ctypes.POINTER(ctypes.c_int)]),
    "swe_lc_fit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_ulonglong,
                                  _dp]),
    "swe_lc_gather": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _dp, ctypes.POINTER(ctypes.c_int)]),
    "swe_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libswe_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch is imported first so that the process holds a single HIP
        # runtime (torch's) and torch's streams are valid handles for it
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError("libswe_hip.so is not built (run paper_1705_00614_amd/build.py); "
                              "there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error():
    return load().swe_last_error().decode()


class SweError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_ERRNAME.get(code, code), msg))
        self.code = code


def _check(rc):
    if rc != 0:
        raise SweError(rc, last_error())
    return rc


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def current_stream():
    """The caller's current HIP stream from torch, or None (library stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


def make_params(prm, skip_dry=True, tile=(0, 0), stream=None):
    inlet = prm.get("inlet") or (0, 0, 0, 0)
    p = SweParams()
    p.precision = int(prm.get("precision", 32))
    p.g = prm["g"]
    p.cfl = prm["courant"]
    p.eps = prm["eps"]
    p.dt_max = prm.get("tau_max", 0.0)
    p.dt_min = prm.get("tau_min", 0.0)
    p.nu = prm.get("nu", 0.0)
    p.f_coriolis = prm.get("f_cor", 0.0)
    p.wind_x = prm.get("wind_x", 0.0)
    p.wind_y = prm.get("wind_y", 0.0)
    p.wind_kappa = prm.get("wind_kappa", 0.0)
    p.h_wind = prm.get("h_wind", 0.1)
    p.limiter = int(prm.get("limiter", 0))
    p.skip_dry = int(bool(skip_dry))
    p.tile_x, p.tile_y = int(tile[0]), int(tile[1])
    p.inlet_i0, p.inlet_j0, p.inlet_ni, p.inlet_nj = (int(v) for v in inlet)
    p.q_base = prm.get("q_base", 0.0)
    p.q_peak = prm.get("q_peak", 0.0)
    p.t_peak = prm.get("t_peak", 0.0)
    p.sigma_t = prm.get("sigma_t", 0.0)
    p.stream = stream
    p.sph_displaced = int(prm.get("sph_displaced", 0))
    p.periodic = int(prm.get("periodic", 0))
    return p


def step_noalloc(sc, b, cf, H, Qx, Qy, H1, Qx1, Qy1, t, out=None, stream="torch"):
    """One step of a caller-owned device layer without allocation
    (swe_step_noalloc): the physics of scenario dict `sc`; b, cf, H, Qx, Qy
    and the outputs H1, Qx1, Qy1 (and the optional 5-double `out`) are
    device tensors of the stencil type (torch), row-major (ny, nx).  Queued
    on the stream, not waited for."""
    st = current_stream() if stream == "torch" else stream
    p = make_params(dict(sc["params"]), True, (0, 0), st)
    ptr = lambda a: ctypes.c_void_p(a.data_ptr())
    rc = load().swe_step_noalloc(int(sc["nx"]), int(sc["ny"]), float(sc["h"]), ctypes.byref(p), ptr(b), ptr(cf),
                                 ptr(H), ptr(Qx), ptr(Qy), ptr(H1), ptr(Qx1), ptr(Qy1), float(t),
                                 None if out is None else ptr(out))
    return _check(rc)


def _grid_inputs(sc, skip_dry, tile, precision, st):
    """swe_create's bed and Manning pointers and parameter block for a
    scenario dict, and the arrays they point into (keep them alive)."""
    shp = (int(sc["ny"]), int(sc["nx"]))
    prm = dict(sc["params"])
    if precision is not None:
        prm["precision"] = precision
    p = make_params(prm, skip_dry, tile, st)
    b = _f64(sc["b"], shp)
    nm = _f64(sc.get("n_manning"), shp)
    H0, Qx0, Qy0 = (_f64(sc.get(k), shp) for k in ("H0", "Qx0", "Qy0"))
    solid = sc.get("solid")
    solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    p.solid = None if solid is None else solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    p.H0, p.Qx0, p.Qy0 = _ptr(H0), _ptr(Qx0), _ptr(Qy0)
    return (_ptr(b), _ptr(nm), p), [b, nm, H0, Qx0, Qy0, solid]


def _batch_inputs(scenarios, tile, precision, st):
    """swe_batch_create's arguments for a list of scenario dicts, and the
    arrays they point into."""
    n = len(scenarios)
    nx = (ctypes.c_int * n)(*[int(sc["nx"]) for sc in scenarios])
    ny = (ctypes.c_int * n)(*[int(sc["ny"]) for sc in scenarios])
    dx = (ctypes.c_double * n)(*[float(sc["h"]) for sc in scenarios])
    bs = (_dp * n)()
    nms = (_dp * n)()
    prm = (SweParams * n)()
    keep = []
    for k, sc in enumerate(scenarios):
        (b, nm, p), kp = _grid_inputs(sc, True, tile, precision, st)
        keep += kp
        bs[k], nms[k], prm[k] = b, nm, p
    return (n, nx, ny, dx, bs, nms, prm), keep


def _shape_table(count, tx, ty, ms):
    if count < 0:
        _check(count)
    return [((tx[k], ty[k]), ms[k]) for k in range(min(count, len(ms)))]


def autotune(sc, warmup=8, steps=32, skip_dry=True, precision=None, stream="torch"):
    """Every compiled tile shape of the scenario's precision timed over
    `steps` steps after `warmup` (swe_autotune): [((tile_x, tile_y), ms)],
    fastest first."""
    st = current_stream() if stream == "torch" else stream
    (b, nm, p), keep = _grid_inputs(sc, skip_dry, (0, 0), precision, st)
    tx, ty, ms = (ctypes.c_int * 16)(), (ctypes.c_int * 16)(), (ctypes.c_double * 16)()
    cnt = load().swe_autotune(int(sc["nx"]), int(sc["ny"]), float(sc["h"]), b, nm, ctypes.byref(p), int(warmup),
                              int(steps), 16, tx, ty, ms)
    return _shape_table(cnt, tx, ty, ms)


def autotune_batch(scenarios, warmup=8, steps=32, precision=None, stream="torch"):
    """The same for a batch (swe_batch_autotune)."""
    st = current_stream() if stream == "torch" else stream
    args, keep = _batch_inputs(scenarios, (0, 0), precision, st)
    tx, ty, ms = (ctypes.c_int * 16)(), (ctypes.c_int * 16)(), (ctypes.c_double * 16)()
    cnt = load().swe_batch_autotune(*args, int(warmup), int(steps), 16, tx, ty, ms)
    return _shape_table(cnt, tx, ty, ms)


class Solver:
    """A GPU solver handle built from a scenario dict (keys nx, ny, h, b,
    n_manning, solid, H0, Qx0, Qy0, params)."""

    def __init__(self, sc, skip_dry=True, tile=(0, 0), precision=None, stream="torch"):
        L = load()
        self.nx, self.ny, self.h = int(sc["nx"]), int(sc["ny"]), float(sc["h"])
        # the cap on every step (0: none), which bounds how far a run can go
        self.tau_max = float(sc["params"].get("tau_max", 0.0))
        st = current_stream() if stream == "torch" else stream
        (b, nm, p), keep = _grid_inputs(sc, skip_dry, tile, precision, st)
        self._h = L.swe_create(self.nx, self.ny, self.h, b, nm, ctypes.byref(p))
        if not self._h:
            raise SweError(SWE_EINVAL, last_error())
        if sc.get("sigma") is not None:
            self.set_source_field(sc["sigma"])

    def close(self):
        if getattr(self, "_h", None):
            load().swe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except TypeError:   # at interpreter exit the module's globals may already be gone
            pass

    def step(self):
        return _check(load().swe_step(self._h))

    def run(self, n):
        return _check(load().swe_run(self._h, int(n)))

    def run_rc(self, n):
        return load().swe_run(self._h, int(n))

    def enqueue(self, n):
        """Queue n steps on the stream without waiting (swe_enqueue)."""
        return _check(load().swe_enqueue(self._h, int(n)))

    def run_timed(self, n):
        ms = ctypes.c_double(0.0)
        _check(load().swe_run_timed(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    def mass(self):
        return load().swe_mass(self._h)

    def time(self):
        return load().swe_time(self._h)

    def last_dt(self):
        return load().swe_last_dt(self._h)

    def next_dt(self):
        return load().swe_next_dt(self._h)

    def ledger(self):
        return load().swe_ledger(self._h)

    def inflow(self):
        return load().swe_inflow(self._h)

    def steps(self):
        return load().swe_steps(self._h)

    def state(self):
        shp = (self.ny, self.nx)
        H, Qx, Qy = (np.empty(shp) for _ in range(3))
        _check(load().swe_get_state(self._h, _ptr(H), _ptr(Qx), _ptr(Qy)))
        return H, Qx, Qy

    def set_state(self, H, Qx=None, Qy=None):
        shp = (self.ny, self.nx)
        H, Qx, Qy = (_f64(a, shp) for a in (H, Qx, Qy))
        return _check(load().swe_set_state(self._h, _ptr(H), _ptr(Qx), _ptr(Qy)))

    def set_time(self, t):
        return _check(load().swe_set_time(self._h, float(t)))

    def work(self):
        t, c = ctypes.c_longlong(), ctypes.c_longlong()
        n, tx, ty = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().swe_work(self._h, ctypes.byref(t), ctypes.byref(c), ctypes.byref(n),
                               ctypes.byref(tx), ctypes.byref(ty)))
        return dict(tile_steps=t.value, cell_steps=c.value, ntiles=n.value, tile=(tx.value, ty.value))

    def set_source_field(self, sigma):
        """Source rate field sigma(x, y) [m/s] (ny, nx), or None to remove it."""
        if sigma is None:
            _check(load().swe_set_source_field(self._h, None))
        else:
            a = _f64(sigma, (self.ny, self.nx))
            _check(load().swe_set_source_field(self._h, _ptr(a)))

    def field_volume(self):
        return load().swe_field_volume(self._h)

    def launch_grid(self):
        """Workgroups of one step launch."""
        n = load().swe_launch_grid(self._h)
        if n < 0:
            raise SweError(n, last_error())
        return n

    def set_launch_grid(self, grid):
        """Workgroups of the following step launches, 8 up to the default
        (swe_set_launch_grid): places the tiles, changes no result."""
        return _check(load().swe_set_launch_grid(self._h, int(grid)))

    def active_tiles(self):
        n = self.work()["ntiles"]
        buf = (ctypes.c_int * max(n, 1))()
        cnt = load().swe_active_tiles(self._h, buf, n)
        if cnt < 0:
            _check(cnt)
        return np.sort(np.array(buf[:cnt], dtype=np.int64))

    def hold_dt(self, tau):
        """Hold the step length at tau from the next step on (0 releases)."""
        _check(load().swe_hold_dt(self._h, float(tau)))

    def enable_line_taps(self, r):
        self.tap_r = int(r)
        _check(load().swe_enable_line_taps(self._h, self.tap_r))

    def zero_line_taps(self):
        _check(load().swe_zero_line_taps(self._h))

    def line_taps(self):
        r = self.tap_r
        tx = np.empty((3, self.ny, self.nx // r + 1))
        ty = np.empty((3, self.ny // r + 1, self.nx))
        _check(load().swe_get_line_taps(self._h, _ptr(tx), _ptr(ty)))
        return tx, ty

    def restrict_from(self, fine, r):
        """This (coarse) grid's layer = r x r means of fine's layer."""
        _check(load().swe_restrict(fine._h, self._h, int(r)))

    def set_correction_depth(self, hmin):
        _check(load().swe_set_correction_depth(self._h, float(hmin)))

    def set_correction(self, dE, dN):
        """Flux corrections (3, ny, nx) through the east and north faces, or None."""
        if dE is None and dN is None:
            _check(load().swe_set_correction(self._h, None, None))
            return
        shp = (3, self.ny, self.nx)
        dE = _f64(np.zeros(shp) if dE is None else dE, shp)
        dN = _f64(np.zeros(shp) if dN is None else dN, shp)
        _check(load().swe_set_correction(self._h, _ptr(dE), _ptr(dN)))


class Batch:
    """Scenarios of uneven grid sizes advanced together by one launch per step
    (``swe_batch_*``).  Each scenario is a dict as for :class:`Solver`;
    precision, limiter and tile shape come from the first one."""

    def __init__(self, scenarios, tile=(0, 0), precision=None, stream="torch"):
        if any(sc.get("sigma") is not None for sc in scenarios):
            raise ValueError("scenarios of a batch carry no source rate field")
        L = load()
        st = current_stream() if stream == "torch" else stream
        self.shapes = [(int(sc["ny"]), int(sc["nx"])) for sc in scenarios]
        args, keep = _batch_inputs(scenarios, tile, precision, st)
        self.n = len(scenarios)
        self._h = L.swe_batch_create(*args)
        if not self._h:
            raise SweError(SWE_EINVAL, last_error())

    def close(self):
        if getattr(self, "_h", None):
            load().swe_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except TypeError:   # at interpreter exit the module's globals may already be gone
            pass

    def run(self, n):
        return _check(load().swe_batch_run(self._h, int(n)))

    def run_rc(self, n):
        return load().swe_batch_run(self._h, int(n))

    def run_timed(self, n):
        ms = ctypes.c_double(0.0)
        _check(load().swe_batch_run_timed(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    def query(self):
        n = self.n
        t, m, q, l = (np.empty(n) for _ in range(4))
        st = (ctypes.c_long * n)()
        _check(load().swe_batch_query(self._h, _ptr(t), _ptr(m), _ptr(q), _ptr(l), st))
        return dict(time=t, mass=m, inflow=q, ledger=l, steps=np.array(st[:], dtype=np.int64))

    def state(self, k):
        shp = self.shapes[k]
        H, Qx, Qy = (np.empty(shp) for _ in range(3))
        _check(load().swe_batch_get_state(self._h, int(k), _ptr(H), _ptr(Qx), _ptr(Qy)))
        return H, Qx, Qy

    def work(self):
        t, c, n = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
        _check(load().swe_batch_work(self._h, ctypes.byref(t), ctypes.byref(c), ctypes.byref(n)))
        return dict(tile_steps=t.value, cell_steps=c.value, total_tiles=n.value)


class Nest:
    """Coarse grid with refined patches (``swe_nest_*``), from a dict with
    keys coarse (scenario dict), patches (dicts with ci0, cj0, cw, ch and the
    extended fine b, n_manning, interior H0, Qx0, Qy0) and r."""

    def __init__(self, nest, feedback=True, precision=None, skip_dry=True, stream="torch"):
        if nest["coarse"].get("sigma") is not None:
            raise ValueError("a nest carries no source rate field")
        L = load()
        sc, r = nest["coarse"], int(nest["r"])
        st = current_stream() if stream == "torch" else stream
        pr = dict(sc["params"])
        if precision is not None:
            pr["precision"] = precision
        p = make_params(pr, skip_dry, (0, 0), st)
        self.shape = (int(sc["ny"]), int(sc["nx"]))
        self.r = r
        # the cap on every coarse step (0: none), which bounds how far a run can go
        self.tau_max = float(pr.get("tau_max", 0.0))
        b = _f64(sc["b"], self.shape)
        nm = _f64(sc.get("n_manning"), self.shape)
        H0, Qx0, Qy0 = (_f64(sc.get(q), self.shape) for q in ("H0", "Qx0", "Qy0"))
        solid = sc.get("solid")
        solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
        p.solid = None if solid is None else solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        p.H0, p.Qx0, p.Qy0 = _ptr(H0), _ptr(Qx0), _ptr(Qy0)
        keep = [b, nm, H0, Qx0, Qy0, solid]
        pats = nest["patches"]
        arr = (SwePatch * len(pats))()
        self.pshapes = []
        for k, q in enumerate(pats):
            cw, ch = int(q["cw"]), int(q["ch"])
            ext = (r * ch + 2 * NEST_FRAME, r * cw + 2 * NEST_FRAME)
            inner = (r * ch, r * cw)
            fb = _f64(q["b"], ext)
            fn = _f64(q.get("n_manning"), ext)
            fH, fX, fY = (_f64(q.get(f), inner) for f in ("H0", "Qx0", "Qy0"))
            keep += [fb, fn, fH, fX, fY]
            arr[k] = SwePatch(int(q["ci0"]), int(q["cj0"]), cw, ch, _ptr(fb), _ptr(fn), _ptr(fH), _ptr(fX),
                              _ptr(fY))
            self.pshapes.append(inner)
        self._h = L.swe_nest_create(self.shape[1], self.shape[0], float(sc["h"]), _ptr(b), _ptr(nm),
                                    ctypes.byref(p), r, 1 if feedback else 0, len(pats),
                                    ctypes.cast(arr, ctypes.c_void_p))
        del keep
        if not self._h:
            raise SweError(SWE_EINVAL, last_error())

    def close(self):
        if getattr(self, "_h", None):
            load().swe_nest_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except TypeError:   # at interpreter exit the module's globals may already be gone
            pass

    def run(self, n):
        return _check(load().swe_nest_run(self._h, int(n)))

    def run_rc(self, n):
        return load().swe_nest_run(self._h, int(n))

    def run_timed(self, n):
        ms = ctypes.c_double(0.0)
        _check(load().swe_nest_run_timed(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    def hold_dt(self, tau_c):
        """Hold the coarse step at tau_c (substeps tau_c / r); 0 returns to the CFL rule."""
        _check(load().swe_nest_hold_dt(self._h, float(tau_c)))

    def time(self):
        return self.query()["time"]

    def next_dt(self):
        """Length of the next coarse step."""
        return self.query()["dt_coarse"]

    def step(self):
        return self.run(1)

    def query(self):
        v = [ctypes.c_double() for _ in range(6)]
        st = ctypes.c_long()
        _check(load().swe_nest_query(self._h, ctypes.byref(v[0]), ctypes.byref(v[1]), ctypes.byref(v[2]),
                                     ctypes.byref(v[3]), ctypes.byref(st), ctypes.byref(v[4]),
                                     ctypes.byref(v[5])))
        return dict(time=v[0].value, volume=v[1].value, inflow=v[2].value, ledger=v[3].value,
                    steps=st.value, dt_coarse=v[4].value, dt_fine=v[5].value)

    def coarse_state(self):
        H, Qx, Qy = (np.empty(self.shape) for _ in range(3))
        _check(load().swe_nest_get_coarse(self._h, _ptr(H), _ptr(Qx), _ptr(Qy)))
        return H, Qx, Qy

    def work(self):
        c, f = ctypes.c_longlong(), ctypes.c_longlong()
        _check(load().swe_nest_work(self._h, ctypes.byref(c), ctypes.byref(f)))
        return dict(coarse_cells=c.value, fine_cells=f.value)

    def patch_state(self, k):
        shp = self.pshapes[k]
        H, Qx, Qy = (np.empty(shp) for _ in range(3))
        _check(load().swe_nest_get_patch(self._h, int(k), _ptr(H), _ptr(Qx), _ptr(Qy)))
        return H, Qx, Qy


LC_LAYERS = ((6, 32), (32, 32), (32, 32), (32, 6))


def lc_pack(W, b):
    """Packed parameter vector from per-layer W (out, in, 3, 3) and b (out)."""
    return np.concatenate([np.concatenate([np.asarray(w, np.float64).ravel(), np.asarray(v, np.float64).ravel()])
                           for w, v in zip(W, b)])


def lc_unpack(p):
    W, b, k = [], [], 0
    for ci, co in LC_LAYERS:
        n = co * ci * 9
        W.append(p[k:k + n].reshape(co, ci, 3, 3))
        k += n
        b.append(p[k:k + co].copy())
        k += co
    return W, b


class Net:
    """The learned flux-correction network (``swe_lc_*``) for tiles of S cells."""

    def __init__(self, tile, max_crops, in_scale, out_scale, stream="torch"):
        L = load()
        st = current_stream() if stream == "torch" else stream
        self.S = int(tile)
        self.So = self.S + 1            # outputs: the tile and the cell row and column before it
        self.in_scale = np.ascontiguousarray(in_scale, dtype=np.float64)
        self.out_scale = np.ascontiguousarray(out_scale, dtype=np.float64)
        self._h = L.swe_lc_create(self.S, int(max_crops), _ptr(self.in_scale), _ptr(self.out_scale), st)
        if not self._h:
            raise SweError(SWE_EINVAL, last_error())
        self.nparams = L.swe_lc_nparams()

    def close(self):
        if getattr(self, "_h", None):
            load().swe_lc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except TypeError:   # at interpreter exit the module's globals may already be gone
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        assert p.shape == (self.nparams,)
        _check(load().swe_lc_set_params(self._h, _ptr(p)))

    def params(self):
        p = np.empty(self.nparams)
        _check(load().swe_lc_get_params(self._h, _ptr(p)))
        return p

    def grads(self):
        p = np.empty(self.nparams)
        _check(load().swe_lc_get_grads(self._h, _ptr(p)))
        return p

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = x.shape[0]
        out = np.empty((n, self.So, self.So, 6))
        _check(load().swe_lc_forward(self._h, n, _ptr(x), _ptr(out)))
        return out

    def infer(self, x):
        """Network output through the one-launch inference path (the one run
        before each step of an attached grid)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = x.shape[0]
        out = np.empty((n, self.So, self.So, 6))
        _check(load().swe_lc_infer(self._h, n, _ptr(x), _ptr(out)))
        return out

    def train_step(self, x, y, mask, lr):
        x, y, mask = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, mask))
        loss = ctypes.c_double()
        _check(load().swe_lc_train_step(self._h, x.shape[0], _ptr(x), _ptr(y), _ptr(mask), float(lr),
                                        ctypes.byref(loss)))
        return loss.value

    def attach(self, solver):
        """Correct every later step of `solver` with this network (None detaches)."""
        if solver is None:
            raise ValueError("use detach(solver)")
        _check(load().swe_lc_attach(self._h, solver._h))

    @staticmethod
    def detach(solver):
        _check(load().swe_lc_attach(None, solver._h))

    def gather(self, solver):
        """Crops (n, S+9, S+9, 6) of the solver's active tiles and their tile indices."""
        nt = solver.work()["ntiles"]
        x = np.empty((nt, self.So + 8, self.So + 8, 6))
        tiles = (ctypes.c_int * nt)()
        n = load().swe_lc_gather(self._h, solver._h, _ptr(x), tiles)
        if n < 0:
            _check(n)
        return x[:n], np.array(tiles[:n], dtype=np.int64)

    def set_out_scale(self, scale):
        self.out_scale = np.ascontiguousarray(scale, dtype=np.float64)
        _check(load().swe_lc_set_out_scale(self._h, _ptr(self.out_scale)))

    def data(self, capacity):
        _check(load().swe_lc_data(self._h, int(capacity)))

    def data_count(self):
        return load().swe_lc_data_count(self._h)

    def collect(self, fine, coarse, r, m):
        """Add one coarse interval of training crops; returns its tau_c."""
        tau = ctypes.c_double()
        _check(load().swe_lc_collect(self._h, fine._h, coarse._h, int(r), int(m), ctypes.byref(tau)))
        return tau.value

    def get_data(self, first, n):
        So = self.So
        x = np.empty((n, So + 8, So + 8, 6))
        y = np.empty((n, So, So, 6))
        m = np.empty((n, So, So, 6))
        t = (ctypes.c_int * max(n, 1))()
        _check(load().swe_lc_get_data(self._h, int(first), int(n), _ptr(x), _ptr(y), _ptr(m), t))
        return x, y, m, np.array(t[:n], dtype=np.int64)

    def fit(self, iters, batch, lr, seed=0):
        losses = np.empty(max(int(iters), 1))
        _check(load().swe_lc_fit(self._h, int(iters), int(batch), float(lr), int(seed), _ptr(losses)))
        return losses[:iters]

    def layer(self, which, n):
        """Stored bf16 values of the last forward/backward (see swe_lc_get_layer)."""
        l = which % 4
        if which < 4:
            side, c = self.So + 8 - 2 * l, LC_LAYERS[l][0]
        else:
            side, c = self.So + 6 - 2 * l, LC_LAYERS[l][1]
        out = np.empty((n, side, side, c))
        _check(load().swe_lc_get_layer(self._h, int(which), _ptr(out)))
        return out
