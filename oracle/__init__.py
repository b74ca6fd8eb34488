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
  gcc ``-O2 -ffp-contract=off -fopenmp``: the loops over rows, columns and
  cells are shared among threads (:func:`set_threads`) with results that are
  bit for bit the same for any thread count.
* ``poisson_oracle.c`` -- plain C: the potential of Sect. 2.1 by red-black
  successive over-relaxation in (r, z), reflecting axis and plane, Roche
  outer values; the acceleration -grad Phi.
* ``levelset_oracle.c`` -- plain C: the level-set flame front of Sect. 2.3,
  advection of the corner field by Hamilton-Jacobi WENO5 with a global LF
  flux and SSP-RK3, and re-distancing (front points by linear interpolation,
  brute-force nearest distance, tanh blend).
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
_SRCS = [os.path.join(_HERE, f) for f in ("hydro_oracle.c", "poisson_oracle.c", "levelset_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

PERIODIC, TRANSMISSIVE, REFLECTING = 0, 1, 2
CARTESIAN, CYLINDRICAL = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle's C sources into ``liboracle.so`` next to them."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, *_SRCS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _PoissonParams(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("rmax", ctypes.c_double), ("zmax", ctypes.c_double),
                ("G", ctypes.c_double), ("mass", ctypes.c_double),
                ("omega", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32)]


class _LsParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("xlo", ctypes.c_double), ("xhi", ctypes.c_double),
                ("ylo", ctypes.c_double), ("yhi", ctypes.c_double),
                ("bc", ctypes.c_int32 * 4), ("eps", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("xlo", ctypes.c_double), ("xhi", ctypes.c_double),
        ("ylo", ctypes.c_double), ("yhi", ctypes.c_double),
        ("geometry", ctypes.c_int32), ("bc", ctypes.c_int32 * 4),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("eps", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
        ("recon", ctypes.c_int32),
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
        lib.orc_weno5_face.restype = ctypes.c_double
        lib.orc_weno5_face.argtypes = [ctypes.c_double] * 11
        lib.orc_alpha.argtypes = [pp, dp, dp]
        lib.orc_cfl.argtypes = [pp, dp, dp]
        lib.orc_rhs.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_step.argtypes = [pp, dp, dp, ctypes.c_double, dp, dp]
        lib.orc_run.argtypes = [pp, dp, dp, ctypes.c_int, ctypes.c_double, dp, dp, dp]
        lib.orc_sums.argtypes = [pp, dp, dp]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        for f in ("orc_alpha", "orc_cfl", "orc_rhs", "orc_step", "orc_run", "orc_sums",
                  "orc_params_size", "orc_set_threads"):
            getattr(lib, f).restype = ctypes.c_int
        assert lib.orc_params_size() == ctypes.sizeof(_Params)
        lib.orc_char_eig.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, dp, dp]
        lib.orc_char_eig.restype = ctypes.c_int
        lib.orc_poisson.argtypes = [ctypes.POINTER(_PoissonParams), dp, dp, dp]
        lib.orc_poisson.restype = ctypes.c_int
        lib.orc_gravity.argtypes = [ctypes.POINTER(_PoissonParams), dp, dp]
        lib.orc_gravity.restype = None
        lib.orc_poisson_params_size.restype = ctypes.c_int
        assert lib.orc_poisson_params_size() == ctypes.sizeof(_PoissonParams)
        lp = ctypes.POINTER(_LsParams)
        lib.orc_ls_alpha.argtypes = [lp, dp, ctypes.c_double, dp]
        lib.orc_ls_alpha.restype = None
        lib.orc_ls_rhs.argtypes = [lp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_ls_rhs.restype = None
        lib.orc_ls_step.argtypes = [lp, dp, dp, ctypes.c_double, ctypes.c_double]
        lib.orc_ls_step.restype = None
        lib.orc_ls_front.argtypes = [lp, dp, dp, ctypes.c_long]
        lib.orc_ls_front.restype = ctypes.c_long
        lib.orc_ls_redistance.argtypes = [lp, dp, dp]
        lib.orc_ls_redistance.restype = ctypes.c_long
        lib.orc_ls_corner_velocity.argtypes = [lp, dp, dp]
        lib.orc_ls_corner_velocity.restype = None
        lib.orc_ls_params_size.restype = ctypes.c_int
        assert lib.orc_ls_params_size() == ctypes.sizeof(_LsParams)
        _lib = lib
    return _lib


def set_threads(n: int) -> int:
    """Threads for the hydro oracle's parallel loops (n >= 1); returns the
    number in effect.  The default is OpenMP's (OMP_NUM_THREADS, else every
    core).  Results do not depend on it."""
    return int(_load().orc_set_threads(int(n)))


def threads() -> int:
    """Threads the hydro oracle's parallel loops use now."""
    return int(_load().orc_set_threads(0))


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


def char_eig(Ul, Ur, direction, gamma):
    """(L, R) (4x4 each) of the characteristic reconstruction at the Roe
    average of two conserved states, in the rotated frame (rho, m_n, m_t, E)."""
    Ul = np.ascontiguousarray(Ul, dtype=np.float64)
    Ur = np.ascontiguousarray(Ur, dtype=np.float64)
    L = np.zeros(16)
    R = np.zeros(16)
    _chk(_load().orc_char_eig(_ptr(Ul), _ptr(Ur), int(direction), float(gamma), _ptr(L), _ptr(R)))
    return L.reshape(4, 4), R.reshape(4, 4)


def weno5(v, eps=1e-6):
    """Scalar WENO5-JS reconstruction at the right face of v[2]."""
    v = [float(x) for x in v]
    return _load().orc_weno5(*v, float(eps))


def weno5_face(p, m, eps=1e-6):
    """Face value: left-biased reconstruction of p[0..4] plus right-biased of
    m[0..4] (m in upwind order, m[0] farthest), over a common denominator."""
    v = [float(x) for x in p] + [float(x) for x in m]
    return _load().orc_weno5_face(*v, float(eps))


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
        p.recon = int(params.get("recon", 0))
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


def _poisson_params(nr, nz, rmax, zmax, G, mass, omega=1.9, tol=1e-8, max_iter=100000):
    q = _PoissonParams()
    q.nr, q.nz = int(nr), int(nz)
    q.rmax, q.zmax = float(rmax), float(zmax)
    q.G, q.mass = float(G), float(mass)
    q.omega, q.tol, q.max_iter = float(omega), float(tol), int(max_iter)
    return q


def poisson(rho, rmax, zmax, G, mass, phi0=None, omega=1.9, tol=1e-8, max_iter=100000):
    """Potential of density rho ((nz, nr), quarter plane r, z >= 0) by red-black
    SOR from phi0 (default 0).  Returns (phi, iterations, last relative change)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    nz, nr = rho.shape
    phi = np.zeros_like(rho) if phi0 is None else np.array(phi0, dtype=np.float64, copy=True)
    q = _poisson_params(nr, nz, rmax, zmax, G, mass, omega, tol, max_iter)
    ch = np.zeros(1)
    it = _load().orc_poisson(ctypes.byref(q), _ptr(rho), _ptr(phi), _ptr(ch))
    if it < 0:
        raise OracleError("poisson: invalid parameters")
    return phi, it, float(ch[0])


def gravity_from_potential(phi, rmax, zmax, G, mass):
    """-grad phi at the cell centres, (2, nz, nr) = (g_r, g_z)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, nr = phi.shape
    q = _poisson_params(nr, nz, rmax, zmax, G, mass)
    g = np.zeros((2, nz, nr))
    _load().orc_gravity(ctypes.byref(q), _ptr(phi), _ptr(g))
    return g


class LevelSet:
    """The level-set oracle on the corners of a grid.

    ``params`` uses the keys nx, ny, xlo, xhi, ylo, yhi, bc (4 ints) and eps of
    the fluid's parameters.  Fields are float64 arrays of shape (ny+1, nx+1);
    corner velocities (2, ny+1, nx+1)."""

    def __init__(self, params: dict):
        q = _LsParams()
        q.nx, q.ny = int(params["nx"]), int(params["ny"])
        q.xlo, q.xhi = float(params["xlo"]), float(params["xhi"])
        q.ylo, q.yhi = float(params["ylo"]), float(params["yhi"])
        for k, b in enumerate(params["bc"]):
            q.bc[k] = int(b)
        q.eps = float(params.get("eps", 1e-6))
        self._q = q
        self.shape = (q.ny + 1, q.nx + 1)
        self._lib = _load()

    def _f(self, S):
        S = np.ascontiguousarray(S, dtype=np.float64)
        assert S.shape == self.shape, S.shape
        return S

    def _v(self, vel):
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        assert vel.shape == (2,) + self.shape, vel.shape
        return vel

    def corner_velocity(self, U):
        """Corner velocity (2, ny+1, nx+1) from a cell state (4, ny, nx)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (4, self.shape[0] - 1, self.shape[1] - 1), U.shape
        vel = np.empty((2,) + self.shape)
        self._lib.orc_ls_corner_velocity(ctypes.byref(self._q), _ptr(U), _ptr(vel))
        return vel

    def alpha(self, vel, s_f=0.0):
        out = np.zeros(2)
        self._lib.orc_ls_alpha(ctypes.byref(self._q), _ptr(self._v(vel)), float(s_f), _ptr(out))
        return out

    def rhs(self, S, vel, s_f, ax, ay):
        S = self._f(S)
        L = np.empty_like(S)
        self._lib.orc_ls_rhs(ctypes.byref(self._q), _ptr(S), _ptr(self._v(vel)), float(s_f),
                             float(ax), float(ay), _ptr(L))
        return L

    def step(self, S, vel, s_f, dt):
        S = self._f(S).copy()
        self._lib.orc_ls_step(ctypes.byref(self._q), _ptr(S), _ptr(self._v(vel)), float(s_f), float(dt))
        return S

    def front(self, S):
        """Front points, (n, 2) = (x, y), in the oracle's order."""
        S = self._f(S)
        cap = 3 * S.size
        pts = np.zeros((cap, 2))
        n = self._lib.orc_ls_front(ctypes.byref(self._q), _ptr(S), _ptr(pts), cap)
        return pts[:n].copy()

    def distance_at(self, S, js, is_):
        """Nearest-front distance of the corners (js[k], is_[k]) by brute force over
        this oracle's front points (the same operations as the C routine)."""
        pts = self.front(S)
        q = self._q
        dx = (q.xhi - q.xlo) / q.nx
        dy = (q.yhi - q.ylo) / q.ny
        x = q.xlo + np.asarray(is_, dtype=np.float64) * dx
        y = q.ylo + np.asarray(js, dtype=np.float64) * dy
        ex = x[:, None] - pts[None, :, 0]
        ey = y[:, None] - pts[None, :, 1]
        return np.sqrt(ex * ex + ey * ey).min(axis=1)

    def redistance(self, S):
        """Returns (S_new, d, number of front points); d is None without front points."""
        S = self._f(S).copy()
        d = np.full_like(S, np.nan)
        n = self._lib.orc_ls_redistance(ctypes.byref(self._q), _ptr(S), _ptr(d))
        return S, (d if n > 0 else None), int(n)
