"""FP64 CPU oracle of the WENO5 / global-LF / SSP-RK3 hydro update.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (the HIP library and its binding in ``paper_1507_08549_amd``) never
imports it, and the two share no code.

Contents
--------
* ``hydro_oracle.c`` -- plain C: one SSP-RK3 step of Eq. euler2D (Sect. 2.1)
  with fifth-order finite-difference WENO on a global Lax-Friedrichs split,
  the CFL step of Sect. 5.3, compensated totals.  Built by :func:`build` with
  gcc ``-O2 -ffp-contract=off``.
* :mod:`oracle.torch_ref` -- the same update written with plain PyTorch CPU
  fp64 tensor operations; its autograd gives the exact vector-Jacobian
  product of one step with the time step and LF speeds held fixed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hydro_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PERIODIC, TRANSMISSIVE, REFLECTING = 0, 1, 2
CARTESIAN, CYLINDRICAL = 0, 1


def build(force: bool = True) -> str:
    """Compile ``hydro_oracle.c`` into ``liboracle.so`` next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("xlo", ctypes.c_double), ("xhi", ctypes.c_double),
        ("ylo", ctypes.c_double), ("yhi", ctypes.c_double),
        ("geometry", ctypes.c_int32), ("bc", ctypes.c_int32 * 4),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("eps", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        lib.orc_weno5.restype = ctypes.c_double
        lib.orc_weno5.argtypes = [ctypes.c_double] * 6
        lib.orc_alpha.argtypes = [pp, dp, dp]
        lib.orc_cfl.argtypes = [pp, dp, dp]
        lib.orc_rhs.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_step.argtypes = [pp, dp, dp, ctypes.c_double, dp, dp]
        lib.orc_run.argtypes = [pp, dp, dp, ctypes.c_int, ctypes.c_double, dp, dp, dp]
        lib.orc_sums.argtypes = [pp, dp, dp]
        for f in ("orc_alpha", "orc_cfl", "orc_rhs", "orc_step", "orc_run", "orc_sums",
                  "orc_params_size"):
            getattr(lib, f).restype = ctypes.c_int
        assert lib.orc_params_size() == ctypes.sizeof(_Params)
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    pass


def _chk(rc):
    if rc < 0:
        names = {-1: "invalid argument", -2: "out of memory", -4: "unphysical state (rho<=0 or p<=0)"}
        raise OracleError(f"oracle error {rc}: {names.get(rc, '?')}")
    return rc


def weno5(v, eps=1e-6):
    """Scalar WENO5-JS reconstruction at the right face of v[2]."""
    v = [float(x) for x in v]
    return _load().orc_weno5(*v, float(eps))


class Oracle:
    """The oracle bound to one problem description.

    ``params`` is a dict with keys nx, ny, xlo, xhi, ylo, yhi, geometry, bc (4
    ints: x-low, x-high, y-low, y-high), gamma, cfl, eps, gx, gy, rho_floor,
    p_floor.  States are float64 arrays of shape (4, ny, nx), components
    (rho, m_x, m_y, E).  ``gravity`` is None or (2, ny, nx) (g_x, g_y)."""

    def __init__(self, params: dict, gravity: np.ndarray | None = None):
        self.params = dict(params)
        p = _Params()
        p.nx, p.ny = int(params["nx"]), int(params["ny"])
        p.xlo, p.xhi = float(params["xlo"]), float(params["xhi"])
        p.ylo, p.yhi = float(params["ylo"]), float(params["yhi"])
        p.geometry = int(params.get("geometry", CARTESIAN))
        for k, b in enumerate(params["bc"]):
            p.bc[k] = int(b)
        p.gamma = float(params["gamma"])
        p.cfl = float(params.get("cfl", 0.5))
        p.eps = float(params.get("eps", 1e-6))
        p.gx, p.gy = float(params.get("gx", 0.0)), float(params.get("gy", 0.0))
        p.rho_floor = float(params.get("rho_floor", 0.0))
        p.p_floor = float(params.get("p_floor", 0.0))
        self._p = p
        self.nx, self.ny = p.nx, p.ny
        self.gravity = None
        if gravity is not None:
            self.gravity = np.ascontiguousarray(gravity, dtype=np.float64)
            assert self.gravity.shape == (2, p.ny, p.nx)
        self._lib = _load()

    def _state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (4, self.ny, self.nx), U.shape
        return U

    def alpha(self, U):
        """(alpha_x, alpha_y, s_max) of a state."""
        U = self._state(U)
        out = np.zeros(3)
        _chk(self._lib.orc_alpha(ctypes.byref(self._p), _ptr(U), _ptr(out)))
        return out

    def cfl(self, U):
        U = self._state(U)
        dt = np.zeros(1)
        _chk(self._lib.orc_cfl(ctypes.byref(self._p), _ptr(U), _ptr(dt)))
        return float(dt[0])

    def rhs(self, U, ax, ay):
        U = self._state(U)
        L = np.empty_like(U)
        _chk(self._lib.orc_rhs(ctypes.byref(self._p), _ptr(self.gravity), _ptr(U),
                               float(ax), float(ay), _ptr(L)))
        return L

    def step(self, U, dt, alpha=None):
        """One SSP-RK3 step; returns (U_new, alpha_used[3][2])."""
        U = self._state(U).copy()
        ain = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64).reshape(6)
        aout = np.zeros(6)
        _chk(self._lib.orc_step(ctypes.byref(self._p), _ptr(self.gravity), _ptr(U), float(dt),
                                _ptr(ain), _ptr(aout)))
        return U, aout.reshape(3, 2)

    def run(self, U, nsteps, t_end=0.0, t0=0.0):
        """Advance with the CFL step.  Returns (U, t, dt_rec, alpha_rec)."""
        U = self._state(U).copy()
        t = np.array([float(t0)])
        dts = np.zeros(max(nsteps, 1))
        als = np.zeros((max(nsteps, 1), 3, 2))
        k = _chk(self._lib.orc_run(ctypes.byref(self._p), _ptr(self.gravity), _ptr(U),
                                   int(nsteps), float(t_end), _ptr(t), _ptr(dts), _ptr(als)))
        return U, float(t[0]), dts[:k].copy(), als[:k].copy()

    def sums(self, U):
        U = self._state(U)
        out = np.zeros(4)
        _chk(self._lib.orc_sums(ctypes.byref(self._p), _ptr(U), _ptr(out)))
        return out
