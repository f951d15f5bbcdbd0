"""ctypes wrapper of the FP64 CPU oracle (``liboracle_swe.so``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU product path never imports it.

The oracle computes one CSPH-TVD shallow-water step exactly as written in
``swe_oracle.c`` (arXiv 1705.00614, Sec. 2.1 Eqs. 1-4, Sec. 2.3 stages I-IV,
Sec. 3 kernels K1-K8); this module only marshals arguments.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "swe_oracle.c")
LIB = os.path.join(HERE, "liboracle_swe.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_u8_p = ctypes.POINTER(ctypes.c_uint8)
_c_int_p = ctypes.POINTER(ctypes.c_int)


def build():
    """Compile the oracle with gcc: IEEE FP64, no contraction into FMA."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", LIB, SRC, "-lm"]
    subprocess.check_call(cmd)
    return LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("g", ctypes.c_double), ("courant", ctypes.c_double),
        ("eps", ctypes.c_double), ("tau_max", ctypes.c_double),
        ("tau_min", ctypes.c_double), ("nu", ctypes.c_double),
        ("f_cor", ctypes.c_double), ("wind_x", ctypes.c_double),
        ("wind_y", ctypes.c_double), ("wind_kappa", ctypes.c_double),
        ("h_wind", ctypes.c_double), ("limiter", ctypes.c_int),
        ("periodic", ctypes.c_int), ("in_i0", ctypes.c_int),
        ("in_j0", ctypes.c_int), ("in_ni", ctypes.c_int),
        ("in_nj", ctypes.c_int), ("q_base", ctypes.c_double),
        ("q_peak", ctypes.c_double), ("t_peak", ctypes.c_double),
        ("sigma_t", ctypes.c_double), ("sph_displaced", ctypes.c_int),
    ]


F_GX, F_GY, F_UHX, F_UHY, F_ULX, F_ULY, F_HT, F_QTX, F_QTY, F_GDX, F_GDY = range(11)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 _c_double_p, _c_double_p, _c_u8_p, _c_double_p,
                                 _c_double_p, _c_double_p, ctypes.POINTER(OrcParams)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        for name in ("orc_step", ):
            getattr(L, name).argtypes = [ctypes.c_void_p]
        L.orc_step_tau.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_run.argtypes = [ctypes.c_void_p, ctypes.c_long]
        for name in ("orc_next_tau", "orc_mass", "orc_time", "orc_last_tau",
                     "orc_ledger", "orc_inflow", "orc_field_volume"):
            getattr(L, name).restype = ctypes.c_double
            getattr(L, name).argtypes = [ctypes.c_void_p]
        L.orc_steps.restype = ctypes.c_long
        L.orc_steps.argtypes = [ctypes.c_void_p]
        L.orc_get_state.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p]
        L.orc_set_state.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p]
        L.orc_get_field.argtypes = [ctypes.c_void_p, ctypes.c_int, _c_double_p]
        L.orc_get_faces.argtypes = [ctypes.c_void_p, ctypes.c_int, _c_double_p,
                                    _c_double_p, _c_double_p]
        L.orc_cell_speeds.argtypes = [ctypes.c_void_p, _c_double_p]
        L.orc_set_correction.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p]
        L.orc_set_correction_depth.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_set_source_field.argtypes = [ctypes.c_void_p, _c_double_p]
        L.orc_tau_from_speed.restype = ctypes.c_double
        L.orc_tau_from_speed.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_hydrograph_volume.restype = ctypes.c_double
        L.orc_hydrograph_volume.argtypes = [ctypes.c_double] * 6
        L.orc_tile_flags.argtypes = [ctypes.c_int] * 4 + [_c_double_p, _c_u8_p,
                                                           ctypes.c_double, _c_int_p, _c_int_p]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(_c_double_p)


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == shape, (a.shape, shape)
    return a


def make_params(prm, periodic=False):
    inlet = prm.get("inlet") or (0, 0, 0, 0)
    return OrcParams(
        g=prm["g"], courant=prm["courant"], eps=prm["eps"],
        tau_max=prm.get("tau_max", 0.0), tau_min=prm.get("tau_min", 0.0),
        nu=prm.get("nu", 0.0), f_cor=prm.get("f_cor", 0.0),
        wind_x=prm.get("wind_x", 0.0), wind_y=prm.get("wind_y", 0.0),
        wind_kappa=prm.get("wind_kappa", 0.0), h_wind=prm.get("h_wind", 0.1),
        limiter=prm.get("limiter", 0), periodic=int(periodic),
        in_i0=inlet[0], in_j0=inlet[1], in_ni=inlet[2], in_nj=inlet[3],
        q_base=prm.get("q_base", 0.0), q_peak=prm.get("q_peak", 0.0),
        t_peak=prm.get("t_peak", 0.0), sigma_t=prm.get("sigma_t", 0.0),
        sph_displaced=int(prm.get("sph_displaced", 0)))


class OracleSim:
    """One oracle simulation built from a scenario dict (see the package's
    ``scenarios`` module): keys nx, ny, h, b, n_manning, solid, H0, Qx0, Qy0,
    params."""

    def __init__(self, sc, periodic=False):
        L = lib()
        sigma = sc.get("sigma")
        self.nx, self.ny, self.h = int(sc["nx"]), int(sc["ny"]), float(sc["h"])
        shp = (self.ny, self.nx)
        self._keep = [_f64(sc.get(k), shp) for k in ("b", "n_manning", "H0", "Qx0", "Qy0")]
        solid = sc.get("solid")
        self._solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
        self._prm = make_params(sc["params"], periodic or bool(sc["params"].get("periodic", 0)))
        b, nm, H0, Qx0, Qy0 = self._keep
        self._h = L.orc_create(self.nx, self.ny, self.h, _dp(b), _dp(nm),
                               None if self._solid is None else self._solid.ctypes.data_as(_c_u8_p),
                               _dp(H0), _dp(Qx0), _dp(Qy0), ctypes.byref(self._prm))
        if not self._h:
            raise ValueError("orc_create rejected the scenario")
        if sigma is not None:
            self.set_source_field(sigma)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def step(self, tau=None):
        L = lib()
        rc = L.orc_step(self._h) if tau is None else L.orc_step_tau(self._h, float(tau))
        if rc:
            raise RuntimeError("oracle step failed: %d" % rc)

    def run(self, n):
        rc = lib().orc_run(self._h, int(n))
        if rc:
            raise RuntimeError("oracle run failed: %d" % rc)

    def try_run(self, n):
        return lib().orc_run(self._h, int(n))

    def next_tau(self):
        return lib().orc_next_tau(self._h)

    def cell_speeds(self):
        out = np.empty((self.ny, self.nx))
        lib().orc_cell_speeds(self._h, _dp(out))
        return out

    def set_correction(self, dE, dN):
        """Flux corrections (3, ny, nx) through east and north faces, or None."""
        if dE is None and dN is None:
            rc = lib().orc_set_correction(self._h, None, None)
        else:
            shp = (3, self.ny, self.nx)
            self._corr = [_f64(np.zeros(shp) if a is None else a, shp) for a in (dE, dN)]
            rc = lib().orc_set_correction(self._h, _dp(self._corr[0]), _dp(self._corr[1]))
        if rc:
            raise RuntimeError("orc_set_correction failed: %d" % rc)

    def set_correction_depth(self, hmin):
        if lib().orc_set_correction_depth(self._h, float(hmin)):
            raise ValueError("invalid correction depth")

    def set_source_field(self, sigma):
        """Rate field sigma(x, y) [m/s] (ny, nx) (rain > 0, losses < 0), or None."""
        if sigma is None:
            rc = lib().orc_set_source_field(self._h, None)
        else:
            self._sigma = _f64(sigma, (self.ny, self.nx))
            rc = lib().orc_set_source_field(self._h, _dp(self._sigma))
        if rc:
            raise ValueError("orc_set_source_field rejected the field")

    def field_volume(self):
        return lib().orc_field_volume(self._h)

    def tau_from_speed(self, smax):
        return lib().orc_tau_from_speed(self._h, float(smax))

    def mass(self):
        return lib().orc_mass(self._h)

    def time(self):
        return lib().orc_time(self._h)

    def last_tau(self):
        return lib().orc_last_tau(self._h)

    def ledger(self):
        return lib().orc_ledger(self._h)

    def inflow(self):
        return lib().orc_inflow(self._h)

    def steps(self):
        return lib().orc_steps(self._h)

    def state(self):
        shp = (self.ny, self.nx)
        H, Qx, Qy = (np.empty(shp) for _ in range(3))
        lib().orc_get_state(self._h, _dp(H), _dp(Qx), _dp(Qy))
        return H, Qx, Qy

    def set_state(self, H, Qx, Qy):
        shp = (self.ny, self.nx)
        H, Qx, Qy = (_f64(a, shp) for a in (H, Qx, Qy))
        rc = lib().orc_set_state(self._h, _dp(H), _dp(Qx), _dp(Qy))
        if rc:
            raise ValueError("orc_set_state rejected the state")

    def field(self, which):
        out = np.empty((self.ny, self.nx))
        lib().orc_get_field(self._h, which, _dp(out))
        return out

    def faces(self, d):
        shp = (self.ny, self.nx + 1) if d == 0 else (self.ny + 1, self.nx)
        FH, Fn, Ft = (np.empty(shp) for _ in range(3))
        lib().orc_get_faces(self._h, d, _dp(FH), _dp(Fn), _dp(Ft))
        return FH, Fn, Ft


def hydrograph_volume(q_base, q_peak, t_peak, sigma_t, t, tau):
    return lib().orc_hydrograph_volume(q_base, q_peak, t_peak, sigma_t, t, tau)


def tile_flags(H, tx, ty, eps, source=None):
    H = np.ascontiguousarray(H, dtype=np.float64)
    ny, nx = H.shape
    ntx, nty = -(-nx // tx), -(-ny // ty)
    own = np.zeros(ntx * nty, dtype=np.int32)
    ring = np.zeros(ntx * nty, dtype=np.int32)
    src = None if source is None else np.ascontiguousarray(source, dtype=np.uint8)
    rc = lib().orc_tile_flags(nx, ny, tx, ty, _dp(H),
                              None if src is None else src.ctypes.data_as(_c_u8_p),
                              eps, own.ctypes.data_as(_c_int_p), ring.ctypes.data_as(_c_int_p))
    if rc:
        raise ValueError("orc_tile_flags rejected its arguments")
    return own.reshape(nty, ntx), ring.reshape(nty, ntx)
