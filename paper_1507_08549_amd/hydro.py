"""Python binding of the HIP library (include/hydro.h): argument marshalling only.

Every computation runs in the library's kernels; PyTorch supplies device
memory (float64 CUDA/HIP tensors of shape (4, ny, nx), components
rho, m_x, m_y, E) and the stream.  If the library is not built, or no GPU is
present, constructing a :class:`Solver` raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhydro.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hydro.h")

HYDRO_OK, HYDRO_E_INVALID, HYDRO_E_NOMEM, HYDRO_E_DEVICE, HYDRO_E_UNPHYSICAL, HYDRO_E_STATE = \
    0, -1, -2, -3, -4, -5
PERIODIC, TRANSMISSIVE, REFLECTING = 0, 1, 2
CARTESIAN, CYLINDRICAL = 0, 1
FP64, FP32_BULK = 0, 1
COMPONENTWISE, CHARACTERISTIC = 0, 1


class HydroError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = load().hydro_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")


class UnphysicalError(HydroError):
    pass


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("xlo", ctypes.c_double), ("xhi", ctypes.c_double),
        ("ylo", ctypes.c_double), ("yhi", ctypes.c_double),
        ("geometry", ctypes.c_int32), ("bc", ctypes.c_int32 * 4),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("weno_eps", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
        ("reconstruction", ctypes.c_int32),
    ]


class Alpha(ctypes.Structure):
    _fields_ = [("ax", ctypes.c_double * 3), ("ay", ctypes.c_double * 3)]


_lib = None

#: names of the entry points declared in include/hydro.h
ENTRY_POINTS = ("hydro_create", "hydro_destroy", "hydro_cfl", "hydro_step", "hydro_run",
                "hydro_run_save", "hydro_rhs", "hydro_step_vjp", "hydro_step_save", "hydro_step_vjp_saved",
                "hydro_step_noalloc",
                "hydro_poisson", "hydro_gravity", "hydro_ls_velocity", "hydro_ls_step", "hydro_ls_front",
                "hydro_ls_redistance", "hydro_sums", "hydro_check", "hydro_strerror")


def declared_entry_points(header: str = HEADER):
    """Function names declared in the public header (for the ABI tests)."""
    with open(header) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hydro_[a-z_]+)\s*\(", src)))


def load():
    """Load libhydro.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1507_08549_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.hydro_create.argtypes = [ctypes.POINTER(Params), vp, vp, ctypes.POINTER(vp)]
    lib.hydro_destroy.argtypes = [vp]
    lib.hydro_cfl.argtypes = [vp, vp, dp]
    lib.hydro_step.argtypes = [vp, vp, ctypes.c_double, ctypes.POINTER(Alpha), ctypes.POINTER(Alpha)]
    lib.hydro_run.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_double, dp, vp, vp]
    lib.hydro_run_save.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_double, dp, vp, vp, vp]
    lib.hydro_rhs.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, vp]
    lib.hydro_step_vjp.argtypes = [vp, vp, ctypes.c_double, ctypes.POINTER(Alpha), vp, vp]
    lib.hydro_step_save.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.POINTER(Alpha), vp, vp]
    lib.hydro_step_vjp_saved.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.POINTER(Alpha), vp, vp]
    lib.hydro_step_noalloc.argtypes = [ctypes.POINTER(Params), vp, vp, vp, ctypes.c_double,
                                       ctypes.POINTER(Alpha), vp]
    lib.hydro_poisson.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), dp]
    lib.hydro_gravity.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, vp]
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.hydro_ls_velocity.argtypes = [vp, vp, vp]
    lib.hydro_ls_step.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double]
    lib.hydro_ls_front.argtypes = [vp, vp, vp, ctypes.c_int64, i64p]
    lib.hydro_ls_redistance.argtypes = [vp, vp, vp, i64p]
    lib.hydro_sums.argtypes = [vp, vp, dp]
    lib.hydro_check.argtypes = [vp]
    lib.hydro_strerror.argtypes = [ip]
    lib.hydro_strerror.restype = ctypes.c_char_p
    for f in ENTRY_POINTS:
        if f != "hydro_strerror":
            getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def make_params(prm: dict, precision=FP64) -> Params:
    p = Params()
    p.nx, p.ny = int(prm["nx"]), int(prm["ny"])
    p.xlo, p.xhi, p.ylo, p.yhi = (float(prm[k]) for k in ("xlo", "xhi", "ylo", "yhi"))
    p.geometry = int(prm.get("geometry", CARTESIAN))
    for k, b in enumerate(prm["bc"]):
        p.bc[k] = int(b)
    p.gamma = float(prm["gamma"])
    p.cfl = float(prm.get("cfl", 0.5))
    p.weno_eps = float(prm.get("eps", 1e-6))
    p.precision = int(precision)
    p.gx, p.gy = float(prm.get("gx", 0.0)), float(prm.get("gy", 0.0))
    p.rho_floor = float(prm.get("rho_floor", 0.0))
    p.p_floor = float(prm.get("p_floor", 0.0))
    p.reconstruction = int(prm.get("recon", COMPONENTWISE))
    return p


def _alpha_struct(alpha):
    if alpha is None:
        return None
    a = np.asarray(alpha, dtype=np.float64).reshape(3, 2)
    s = Alpha()
    for k in range(3):
        s.ax[k], s.ay[k] = float(a[k, 0]), float(a[k, 1])
    return s


def _alpha_array(s: Alpha):
    return np.array([[s.ax[k], s.ay[k]] for k in range(3)])


#: largest grid hydro_step_noalloc accepts (nx * ny)
NOALLOC_MAX_CELLS = 1 << 20


def step_noalloc(params: dict, U, dt, alpha=None, gravity=None, precision=FP64, unphysical=None):
    """hydro_step_noalloc: one SSP-RK3 step of U (float64 device tensor (4, ny, nx),
    in place) with no context and no device allocation, on torch's current
    stream.  gravity: None or a (2, ny, nx) float64 device tensor; unphysical:
    None or a one-element int32 device tensor receiving 1 if a stage produced
    rho <= 0 or p <= 0, else 0."""
    import torch
    lib = load()
    nx, ny = int(params["nx"]), int(params["ny"])
    for name, x, shape, dt_ in (("U", U, (4, ny, nx), torch.float64),
                                ("gravity", gravity, (2, ny, nx), torch.float64),
                                ("unphysical", unphysical, (1,), torch.int32)):
        if x is None and name != "U":
            continue
        if (not isinstance(x, torch.Tensor) or x.dtype != dt_ or not x.is_cuda
                or tuple(x.shape) != shape or not x.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dt_} device tensor of shape {shape}")
    p = make_params(params, precision)
    a = _alpha_struct(alpha)
    rc = lib.hydro_step_noalloc(ctypes.byref(p), None if gravity is None else gravity.data_ptr(),
                                torch.cuda.current_stream(U.device).cuda_stream, U.data_ptr(), float(dt),
                                ctypes.byref(a) if a is not None else None,
                                None if unphysical is None else unphysical.data_ptr())
    if rc < 0:
        raise HydroError(rc, "hydro_step_noalloc")


class Solver:
    """One library context: a problem description bound to a device and stream.

    ``params`` is the dict produced by :mod:`paper_1507_08549_amd.inputs`;
    ``gravity`` an optional (2, ny, nx) float64 device tensor (kept alive by
    the solver); ``precision`` FP64 or FP32_BULK."""

    def __init__(self, params: dict, gravity=None, precision=FP64, device=None):
        import torch
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the hydro library runs on the device only")
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self.precision = precision
        self.gravity = None
        gptr = None
        if gravity is not None:
            g = torch.as_tensor(gravity, dtype=torch.float64, device=self.device).contiguous()
            if tuple(g.shape) != (2, self.ny, self.nx):
                raise ValueError(f"gravity must have shape (2, {self.ny}, {self.nx})")
            self.gravity = g
            gptr = g.data_ptr()
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self._p = make_params(params, precision)
            h = ctypes.c_void_p()
            rc = lib.hydro_create(ctypes.byref(self._p), gptr, self.stream.cuda_stream, ctypes.byref(h))
        self._check(rc, "hydro_create")
        self._h = h
        self._lib = lib

    # -- helpers
    def _check(self, rc, where):
        if rc == HYDRO_E_UNPHYSICAL:
            raise UnphysicalError(rc, where)
        if rc < 0:
            raise HydroError(rc, where)
        return rc

    def _state(self, U, name="U"):
        t = self.torch
        if not isinstance(U, t.Tensor) or U.dtype != t.float64 or U.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if tuple(U.shape) != (4, self.ny, self.nx) or not U.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape (4, {self.ny}, {self.nx})")
        return U.data_ptr()

    def new_state(self):
        return self.torch.empty((4, self.ny, self.nx), dtype=self.torch.float64, device=self.device)

    # -- API
    def cfl(self, U) -> float:
        dt = ctypes.c_double()
        self._check(self._lib.hydro_cfl(self._h, self._state(U), ctypes.byref(dt)), "hydro_cfl")
        return dt.value

    def step(self, U, dt, alpha=None, return_alpha=False):
        """One SSP-RK3 step in place.  alpha: None (computed) or (3, 2) speeds."""
        a_in = _alpha_struct(alpha)
        a_out = Alpha() if return_alpha else None
        rc = self._lib.hydro_step(self._h, self._state(U), float(dt),
                                  ctypes.byref(a_in) if a_in is not None else None,
                                  ctypes.byref(a_out) if a_out is not None else None)
        self._check(rc, "hydro_step")
        return _alpha_array(a_out) if return_alpha else None

    def run(self, U, nsteps, t_end=0.0, t0=0.0, record=False):
        """Up to nsteps CFL steps in place.  Returns (steps, t, dt_rec, alpha_rec);
        the records are device tensors (or None)."""
        t = self.torch
        tt = ctypes.c_double(float(t0))
        dts = als = None
        if record:
            dts = t.zeros(max(nsteps, 1), dtype=t.float64, device=self.device)
            als = t.zeros((max(nsteps, 1), 6), dtype=t.float64, device=self.device)
        rc = self._lib.hydro_run(self._h, self._state(U), int(nsteps), float(t_end), ctypes.byref(tt),
                                 dts.data_ptr() if record else None,
                                 als.data_ptr() if record else None)
        k = self._check(rc, "hydro_run")
        if record:
            dts = dts[:k]
            als = als[:k].reshape(k, 2, 3).transpose(1, 2)
        return k, tt.value, dts, als

    def run_into(self, U, nsteps, dt_rec, alpha_rec, t_end=0.0, t0=0.0):
        """hydro_run recording into caller-provided device tensors dt_rec (nsteps,)
        and alpha_rec (nsteps, 6) (ax[0..2], ay[0..2] per step).  Returns steps taken."""
        t = self.torch
        for name, x, shape in (("dt_rec", dt_rec, (nsteps,)), ("alpha_rec", alpha_rec, (nsteps, 6))):
            if (not isinstance(x, t.Tensor) or x.dtype != t.float64 or x.device != self.device
                    or tuple(x.shape) != shape or not x.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 {shape} tensor on {self.device}")
        tt = ctypes.c_double(float(t0))
        rc = self._lib.hydro_run(self._h, self._state(U), int(nsteps), float(t_end), ctypes.byref(tt),
                                 dt_rec.data_ptr(), alpha_rec.data_ptr())
        return self._check(rc, "hydro_run")

    def run_save(self, U, nsteps, states, dt_rec, alpha_rec, t_end=0.0, t0=0.0):
        """hydro_run_save: as run_into, also filling states (nsteps, 3, 4, ny, nx)
        with each step's start state and its two stage states.  Returns steps taken."""
        t = self.torch
        shape = (nsteps, 3, 4, self.ny, self.nx)
        for name, x, shp in (("dt_rec", dt_rec, (nsteps,)), ("alpha_rec", alpha_rec, (nsteps, 6)),
                             ("states", states, shape)):
            if (not isinstance(x, t.Tensor) or x.dtype != t.float64 or x.device != self.device
                    or tuple(x.shape) != shp or not x.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 {shp} tensor on {self.device}")
        tt = ctypes.c_double(float(t0))
        rc = self._lib.hydro_run_save(self._h, self._state(U), int(nsteps), float(t_end), ctypes.byref(tt),
                                      dt_rec.data_ptr(), alpha_rec.data_ptr(), states.data_ptr())
        return self._check(rc, "hydro_run_save")

    def rhs(self, V, ax, ay, out=None):
        L = self.new_state() if out is None else out
        self._check(self._lib.hydro_rhs(self._h, self._state(V), float(ax), float(ay),
                                        self._state(L, "L")), "hydro_rhs")
        return L

    def step_vjp(self, U_n, dt, alpha, lam_next, out=None):
        lam_prev = self.new_state() if out is None else out
        a = _alpha_struct(alpha)
        rc = self._lib.hydro_step_vjp(self._h, self._state(U_n), float(dt), ctypes.byref(a),
                                      self._state(lam_next, "lam_next"), self._state(lam_prev, "lam_prev"))
        self._check(rc, "hydro_step_vjp")
        return lam_prev

    def step_save(self, U, dt, alpha, U1, U2, out=None):
        """One step U -> out (in place if out is None), keeping its stage states in
        U1, U2.  alpha: None or (3, 2) recorded speeds."""
        a_in = _alpha_struct(alpha)
        dst = U if out is None else out
        rc = self._lib.hydro_step_save(self._h, self._state(U), self._state(dst, "out"), float(dt),
                                       ctypes.byref(a_in) if a_in is not None else None,
                                       self._state(U1, "U1"), self._state(U2, "U2"))
        self._check(rc, "hydro_step_save")
        return dst

    def step_vjp_saved(self, U_n, U1, U2, dt, alpha, lam_next, out=None):
        lam_prev = self.new_state() if out is None else out
        a = _alpha_struct(alpha)
        rc = self._lib.hydro_step_vjp_saved(self._h, self._state(U_n), self._state(U1, "U1"),
                                            self._state(U2, "U2"), float(dt), ctypes.byref(a),
                                            self._state(lam_next, "lam_next"),
                                            self._state(lam_prev, "lam_prev"))
        self._check(rc, "hydro_step_vjp_saved")
        return lam_prev

    def _field(self, x, name, ncomp):
        t = self.torch
        if not isinstance(x, t.Tensor) or x.dtype != t.float64 or x.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        shape = (self.ny, self.nx) if ncomp == 1 else (ncomp, self.ny, self.nx)
        if tuple(x.shape) != shape or not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape}")
        return x.data_ptr()

    def poisson(self, rho, phi, G, mass, omega=1.9, tol=1e-8, max_iter=100000):
        """Potential of rho ((ny, nx)) into phi ((ny, nx), in: start, out: solution).
        Returns (iterations, last relative change)."""
        it = ctypes.c_int32()
        ch = ctypes.c_double()
        rc = self._lib.hydro_poisson(self._h, self._field(rho, "rho", 1), self._field(phi, "phi", 1),
                                     float(G), float(mass), float(omega), float(tol), int(max_iter),
                                     ctypes.byref(it), ctypes.byref(ch))
        self._check(rc, "hydro_poisson")
        return it.value, ch.value

    def gravity_from_potential(self, phi, G, mass, out=None):
        """-grad phi, (2, ny, nx); ``out`` may be this solver's own gravity field."""
        g = self.torch.empty((2, self.ny, self.nx), dtype=self.torch.float64, device=self.device) \
            if out is None else out
        rc = self._lib.hydro_gravity(self._h, self._field(phi, "phi", 1), float(G), float(mass),
                                     self._field(g, "g", 2))
        self._check(rc, "hydro_gravity")
        return g

    # -- level set on the (ny+1, nx+1) corners
    def _corner(self, x, name, ncomp=1):
        t = self.torch
        if not isinstance(x, t.Tensor) or x.dtype != t.float64 or x.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        shape = (self.ny + 1, self.nx + 1) if ncomp == 1 else (ncomp, self.ny + 1, self.nx + 1)
        if tuple(x.shape) != shape or not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape}")
        return x.data_ptr()

    def ls_velocity(self, U, out=None):
        """Corner velocity (2, ny+1, nx+1) from a cell state."""
        vel = self.torch.empty((2, self.ny + 1, self.nx + 1), dtype=self.torch.float64,
                               device=self.device) if out is None else out
        rc = self._lib.hydro_ls_velocity(self._h, self._state(U), self._corner(vel, "vel", 2))
        self._check(rc, "hydro_ls_velocity")
        return vel

    def ls_step(self, S, vel, s_flame, dt):
        """One SSP-RK3 step of the level-set advection, S in place."""
        rc = self._lib.hydro_ls_step(self._h, self._corner(S, "S"), self._corner(vel, "vel", 2),
                                     float(s_flame), float(dt))
        self._check(rc, "hydro_ls_step")

    def ls_front(self, S, cap=None):
        """Front points (n, 2) of S, in no particular order."""
        cap = 3 * (self.nx + 1) * (self.ny + 1) if cap is None else int(cap)
        pts = self.torch.empty((max(cap, 1), 2), dtype=self.torch.float64, device=self.device)
        n = ctypes.c_int64()
        rc = self._lib.hydro_ls_front(self._h, self._corner(S, "S"), pts.data_ptr(), cap, ctypes.byref(n))
        self._check(rc, "hydro_ls_front")
        return pts[:min(n.value, cap)]

    def ls_redistance(self, S, dist=None, count=True):
        """Re-distance S in place; returns the number of front points (count=True,
        which waits for the result) or None (count=False: only enqueued)."""
        n = ctypes.c_int64()
        rc = self._lib.hydro_ls_redistance(self._h, self._corner(S, "S"),
                                           None if dist is None else self._corner(dist, "dist"),
                                           ctypes.byref(n) if count else None)
        self._check(rc, "hydro_ls_redistance")
        return n.value if count else None

    def sums(self, U):
        out = (ctypes.c_double * 4)()
        self._check(self._lib.hydro_sums(self._h, self._state(U), out), "hydro_sums")
        return np.array(out[:])

    def check(self):
        return self._check(self._lib.hydro_check(self._h), "hydro_check")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hydro_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
