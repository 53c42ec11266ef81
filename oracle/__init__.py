"""FP64 CPU oracle for the split MUSCL-Hancock / HLLC Euler step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP library.  The arithmetic lives in
``euler_oracle.c``; this module only marshals numpy arrays through ctypes.

Arrays are planar FP64 ``[5, nz, ny, nx]`` (components rho, m_x, m_y, m_z, E),
C-contiguous.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

STAGES = {0: "dt", 1: "input", 2: "extrapolated", 3: "evolved", 4: "output"}


class OracleNonPhysical(RuntimeError):
    """The scheme met rho <= 0, p <= 0 or a non-finite value."""

    def __init__(self, info, step=None):
        self.info = [int(v) for v in info]
        self.step = step
        stage = STAGES.get(self.info[0], str(self.info[0]))
        super().__init__(
            f"non-physical state at step {step}, stage {stage}, axis {self.info[1]}, "
            f"cell (i={self.info[2]}, j={self.info[3]}, k={self.info[4]})")


def load(path=None, rebuild=False):
    """Load liboracle.so (building it first when missing or when asked)."""
    global _LIB
    if path is None:
        if _LIB is not None and not rebuild:
            return _LIB
        path = _build.LIBRARY
        if rebuild or not os.path.exists(path) or \
                os.path.getmtime(path) < os.path.getmtime(_build.SOURCE):
            _build.build()
    lib = ctypes.CDLL(path)
    _declare(lib)
    if path == _build.LIBRARY:
        _LIB = lib
    return lib


def _declare(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_abi_version.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_pressure.argtypes = [dp]
    lib.oracle_pressure.restype = ctypes.c_double
    lib.oracle_flux.argtypes = [dp, ctypes.c_int, dp]
    lib.oracle_prim_to_cons.argtypes = [ctypes.c_int64, dp, dp]
    lib.oracle_cons_to_prim.argtypes = [ctypes.c_int64, dp, dp]
    lib.oracle_minmod.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_minmod.restype = ctypes.c_double
    lib.oracle_hllc.argtypes = [dp, dp, ctypes.c_int, dp]
    lib.oracle_pencil_scratch.argtypes = [ctypes.c_int]
    lib.oracle_pencil_scratch.restype = ctypes.c_int64
    lib.oracle_sweep_pencil.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        dp, dp, dp, ip]
    lib.oracle_sweep_pencil.restype = ctypes.c_int
    lib.oracle_max_wavespeed.argtypes = [ip, dp, dp, i64p]
    lib.oracle_max_wavespeed.restype = ctypes.c_int
    lib.oracle_dt.argtypes = [dp, dp, ctypes.c_double]
    lib.oracle_dt.restype = ctypes.c_double
    lib.oracle_sweep.argtypes = [ip, dp, ip, ctypes.c_int, ctypes.c_double, dp, i64p]
    lib.oracle_sweep.restype = ctypes.c_int
    lib.oracle_run.argtypes = [ip, dp, ip, ip, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int, ctypes.c_double, dp, dp, dp, ip, i64p]
    lib.oracle_run.restype = ctypes.c_int


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(vals, ctype):
    return (ctype * len(vals))(*vals)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


class Oracle:
    """Thin numpy front end over liboracle.so (one instance per library)."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # -- threads ---------------------------------------------------------
    def num_threads(self):
        return int(self.lib.oracle_num_threads())

    def set_num_threads(self, n):
        self.lib.oracle_set_num_threads(int(n))

    # -- point functions -------------------------------------------------
    def pressure(self, U):
        U = _f64(U, (5,))
        return float(self.lib.oracle_pressure(_dptr(U)))

    def flux(self, U, axis):
        U = _f64(U, (5,))
        F = np.zeros(5)
        self.lib.oracle_flux(_dptr(U), int(axis), _dptr(F))
        return F

    def hllc(self, UL, UR, axis):
        UL = _f64(UL, (5,))
        UR = _f64(UR, (5,))
        F = np.zeros(5)
        self.lib.oracle_hllc(_dptr(UL), _dptr(UR), int(axis), _dptr(F))
        return F

    def minmod(self, a, b):
        return float(self.lib.oracle_minmod(float(a), float(b)))

    def prim_to_cons(self, W):
        W = _f64(W)
        U = np.empty_like(W)
        ncell = W.size // 5
        self.lib.oracle_prim_to_cons(ncell, _dptr(W), _dptr(U))
        return U

    def cons_to_prim(self, U):
        U = _f64(U)
        W = np.empty_like(U)
        ncell = U.size // 5
        self.lib.oracle_cons_to_prim(ncell, _dptr(U), _dptr(W))
        return W

    def sweep_pencil(self, W, axis, lam):
        """One pencil update; W is (n+4, 5) with ghost cells filled."""
        W = _f64(W)
        n = W.shape[0] - 4
        out = np.zeros((n, 5))
        scr = np.zeros(int(self.lib.oracle_pencil_scratch(n)))
        bad = ctypes.c_int(0)
        st = self.lib.oracle_sweep_pencil(n, int(axis), float(lam), _dptr(W), _dptr(out),
                                          _dptr(scr), ctypes.byref(bad))
        return out, int(st), int(bad.value)

    # -- grid functions --------------------------------------------------
    def max_wavespeed(self, U):
        U = _f64(U)
        n = _vec([U.shape[3], U.shape[2], U.shape[1]], ctypes.c_int)
        S = np.zeros(3)
        bad = ctypes.c_int64(-1)
        st = self.lib.oracle_max_wavespeed(n, _dptr(U), _dptr(S), ctypes.byref(bad))
        if st != 0:
            raise OracleNonPhysical([0, -1, bad.value, 0, 0, 0], step=0)
        return S

    def dt(self, S, dx, cfl):
        S = _f64(S, (3,))
        dx = _f64(dx, (3,))
        return float(self.lib.oracle_dt(_dptr(S), _dptr(dx), float(cfl)))

    def sweep(self, U, axis, dt, dx, bc):
        """One sweep along `axis` with time step dt; returns a new array."""
        out = np.array(U, dtype=np.float64, copy=True, order="C")
        n = _vec([out.shape[3], out.shape[2], out.shape[1]], ctypes.c_int)
        info = np.full(6, -1, dtype=np.int64)
        st = self.lib.oracle_sweep(n, _dptr(_f64(dx, (3,))), _vec(list(bc), ctypes.c_int),
                                   int(axis), float(dt), _dptr(out),
                                   info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        if st == 1:
            raise OracleNonPhysical(info, step=0)
        if st != 0:
            raise RuntimeError(f"oracle_sweep failed with status {st}")
        return out

    def run(self, U0, nsteps, dx, bc, cfl=0.9, dt_fixed=0.0, t_end=0.0, order=(0, 1, 2)):
        """Advance a copy of U0 by nsteps steps.

        Returns (U, t, dts): final state, time reached and the list of step
        sizes.  Raises OracleNonPhysical when the scheme meets a bad state."""
        U = np.array(U0, dtype=np.float64, copy=True, order="C")
        if U.ndim != 4 or U.shape[0] != 5:
            raise ValueError("state must be [5, nz, ny, nx]")
        n = _vec([U.shape[3], U.shape[2], U.shape[1]], ctypes.c_int)
        dts = np.zeros(max(int(nsteps), 1))
        t = ctypes.c_double(0.0)
        done = ctypes.c_int(0)
        info = np.full(6, -1, dtype=np.int64)
        st = self.lib.oracle_run(n, _dptr(_f64(dx, (3,))), _vec(list(bc), ctypes.c_int),
                                 _vec(list(order), ctypes.c_int), float(cfl), float(dt_fixed),
                                 int(nsteps), float(t_end), _dptr(U), ctypes.byref(t),
                                 _dptr(dts), ctypes.byref(done),
                                 info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        if st == 1:
            raise OracleNonPhysical(info, step=done.value)
        if st != 0:
            raise RuntimeError(f"oracle_run failed with status {st}")
        return U, float(t.value), dts[:done.value].copy()
