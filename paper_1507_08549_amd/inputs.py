"""Seeded synthetic inputs: problem parameters and initial states.

This module is shared by the HIP path's tests and by the oracle's tests.  It
holds no arithmetic of the hydro method itself: it only builds parameter
dicts and initial conserved states (rho, m_x, m_y, E) of shape (4, ny, nx),
sampled at cell centres x_i = xlo + (i + 1/2) dx.

Workloads
---------
* :func:`sod` -- the standard Sod shock tube (1D limit, transmissive).
* :func:`riemann_1d` -- the Riemann problems of Table Test1D (Sect. 5.1).
* :func:`kelvin_helmholtz` -- periodic shear layer with seeded v_y noise.
* :func:`rayleigh_taylor` -- heavy-over-light layer under uniform gravity.
* :func:`polytrope` -- n = 3 Lane-Emden star in (r, z) with a fixed gravity
  field from the enclosed mass (the paper's stars are built in hydrostatic
  equilibrium, Sect. 5.3; here with an ideal gas).
* :func:`kh_sine_amplitudes` / :func:`kh_sine_state` -- the shear layer whose
  v_y is a sum of sine modes, differentiable in the amplitudes (torch).
* :func:`advection_1d`, :func:`advection_2d`, :func:`homologous` -- smooth
  problems with exact solutions, used to pin the oracle.
* :func:`gresho`, :func:`blast`, :func:`explosion` -- the 2D tests of
  Sect. 5.2.

Random draws use ``numpy.random.default_rng(seed)``; ``uniform(-1, 1,
(ny, nx))`` is drawn in C order (row = y).

The benchmark workloads' states are bit-reproducible on any x86-64 host:
their transcendental values come from the C library one value at a time
(:func:`_libm`), not from numpy's vectorised kernels (which differ with the
CPU's vector extensions), and the sine-mode sum runs in a fixed order instead
of through a BLAS product (whose summation order depends on the CPU).
"""
from __future__ import annotations

import functools
import math

import numpy as np

PERIODIC, TRANSMISSIVE, REFLECTING = 0, 1, 2
CARTESIAN, CYLINDRICAL = 0, 1


def _libm(f, a):
    """f (a scalar function of the math module) applied to every element of a."""
    a = np.asarray(a, dtype=np.float64)
    return np.fromiter((f(float(x)) for x in a.ravel()), dtype=np.float64, count=a.size).reshape(a.shape)


def _libm_pow(a, e):
    a = np.asarray(a, dtype=np.float64)
    e = float(e)
    return np.fromiter((math.pow(float(x), e) for x in a.ravel()), dtype=np.float64,
                       count=a.size).reshape(a.shape)


def make_params(nx, ny, xlo, xhi, ylo, yhi, bc, gamma, cfl=0.5, eps=1e-6,
                geometry=CARTESIAN, gx=0.0, gy=0.0, rho_floor=0.0, p_floor=0.0):
    return dict(nx=int(nx), ny=int(ny), xlo=float(xlo), xhi=float(xhi), ylo=float(ylo),
                yhi=float(yhi), bc=[int(b) for b in bc], gamma=float(gamma), cfl=float(cfl),
                eps=float(eps), geometry=int(geometry), gx=float(gx), gy=float(gy),
                rho_floor=float(rho_floor), p_floor=float(p_floor))


def centres(params):
    """Cell-centre coordinates (x of shape (nx,), y of shape (ny,))."""
    nx, ny = params["nx"], params["ny"]
    dx = (params["xhi"] - params["xlo"]) / nx
    dy = (params["yhi"] - params["ylo"]) / ny
    x = params["xlo"] + (np.arange(nx) + 0.5) * dx
    y = params["ylo"] + (np.arange(ny) + 0.5) * dy
    return x, y


def state_from_primitive(rho, u, v, p, gamma):
    """Conserved state from primitive fields (ideal gas, E = p/(gamma-1) + rho |v|^2 / 2)."""
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, u, v, p)))
    U = np.empty((4,) + rho.shape)
    U[0] = rho
    U[1] = rho * u
    U[2] = rho * v
    U[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.ascontiguousarray(U)


def primitive_from_state(U, gamma):
    """(rho, u, v, p) of a conserved state; for plotting and error norms only."""
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


# ----------------------------------------------------------------- 1D tests

def riemann_1d(rho_l, u_l, p_l, rho_r, u_r, p_r, x0=0.5, n=400, gamma=1.4, cfl=0.6):
    """A shock tube on [0, 1] with the split at x0 (the 1D limit: ny = 1)."""
    prm = make_params(n, 1, 0.0, 1.0, 0.0, 1.0, [TRANSMISSIVE] * 4, gamma, cfl)
    x, _ = centres(prm)
    left = x < x0
    rho = np.where(left, rho_l, rho_r)[None, :]
    u = np.where(left, u_l, u_r)[None, :]
    p = np.where(left, p_l, p_r)[None, :]
    return prm, state_from_primitive(rho, u, 0.0, p, gamma)


def sod(n=400, gamma=1.4, cfl=0.6):
    """Standard Sod tube: (1, 0, 1) | (0.125, 0, 0.1) at x = 0.5, run to t = 0.2."""
    return riemann_1d(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 0.5, n, gamma, cfl)


# ----------------------------------------------------------------- 2D tests

def kelvin_helmholtz(n=512, seed=2, gamma=5.0 / 3.0, cfl=0.5, noise=0.01):
    """Periodic unit square: rho = 2, u = +0.5 for |y - 0.5| < 0.25, else rho = 1,
    u = -0.5; p = 2.5; v_y = noise * U(-1, 1) per cell."""
    prm = make_params(n, n, 0.0, 1.0, 0.0, 1.0, [PERIODIC] * 4, gamma, cfl)
    x, y = centres(prm)
    inner = (np.abs(y - 0.5) < 0.25)[:, None] * np.ones((1, n), dtype=bool)
    rho = np.where(inner, 2.0, 1.0)
    u = np.where(inner, 0.5, -0.5)
    rng = np.random.default_rng(seed)
    v = noise * rng.uniform(-1.0, 1.0, (n, n))
    return prm, state_from_primitive(rho, u, v, 2.5, gamma)


def rayleigh_taylor(nx=256, ny=1024, seed=3, gamma=1.4, cfl=0.5, g=-0.1):
    """[0, 0.5] x [0, 2], reflecting walls, uniform gravity g in y; rho = 2 above
    y = 1, 1 below; hydrostatic p with p(1) = 2.5; single-mode v_y seed plus
    1e-4 uniform noise."""
    prm = make_params(nx, ny, 0.0, 0.5, 0.0, 2.0, [REFLECTING] * 4, gamma, cfl, gy=g)
    x, y = centres(prm)
    X, Y = np.meshgrid(x, y)
    rho = np.where(Y > 1.0, 2.0, 1.0)
    p = 2.5 + g * rho * (Y - 1.0)
    rng = np.random.default_rng(seed)
    cx = _libm(math.cos, 4.0 * np.pi * x)[None, :]
    cy = _libm(math.cos, np.pi * (y - 1.0))[:, None]
    v = 0.01 * (1.0 + cx) * (1.0 + cy) / 4.0
    v = v + 1e-4 * rng.uniform(-1.0, 1.0, (ny, nx))
    return prm, state_from_primitive(rho, 0.0, v, p, gamma)


@functools.lru_cache(maxsize=8)
def lane_emden(n, h=1e-4):
    """Integrate theta'' + (2/xi) theta' + theta^n = 0, theta(0) = 1, theta'(0) = 0,
    with classical RK4 in xi (step h) from a series start, up to the first zero.

    Returns (xi, theta, dtheta, xi1): tables on the uniform xi grid ending at the
    last point with theta > 0, and the first zero xi1 (linear interpolation)."""
    n = float(n)

    def rhs(xi, th, ph):
        return ph, -(max(th, 0.0) ** n) - 2.0 * ph / xi

    xi = 10.0 * h
    th = 1.0 - xi ** 2 / 6.0 + n * xi ** 4 / 120.0
    ph = -xi / 3.0 + n * xi ** 3 / 30.0
    xs, ths, phs = [0.0, xi], [1.0, th], [0.0, ph]
    # fill the series start on the table too
    while th > 0.0 and xi < 50.0:
        k1 = rhs(xi, th, ph)
        k2 = rhs(xi + 0.5 * h, th + 0.5 * h * k1[0], ph + 0.5 * h * k1[1])
        k3 = rhs(xi + 0.5 * h, th + 0.5 * h * k2[0], ph + 0.5 * h * k2[1])
        k4 = rhs(xi + h, th + h * k3[0], ph + h * k3[1])
        th_new = th + h / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        ph_new = ph + h / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        if th_new <= 0.0:
            xi1 = xi + h * th / (th - th_new)
            xs_a, th_a, ph_a = np.array(xs), np.array(ths), np.array(phs)
            ph1 = ph + (ph_new - ph) * (xi1 - xi) / h
            return (np.append(xs_a, xi1), np.append(th_a, 0.0), np.append(ph_a, ph1), xi1)
        xi += h
        th, ph = th_new, ph_new
        xs.append(xi)
        ths.append(th)
        phs.append(ph)
    return np.array(xs), np.array(ths), np.array(phs), math.inf


def polytrope(n=1024, seed=4, poly_n=3.0, K=1.0, rho_c=1.0, G=1.0, rho_floor=1e-8,
              extent=1.2, cfl=0.5, noise=1e-3, h=1e-4):
    """n = 3 polytrope in cylindrical (r, z) on the quarter plane [0, 1.2 R]^2.

    gamma = 1 + 1/n, a = sqrt((n+1) K rho_c^(1/n - 1) / (4 pi G)), R = a xi1.
    rho = rho_c theta^n (1 + noise U(-1, 1)) where that exceeds the floor, else
    the floor (no noise); p = K max(rho_LE, floor)^gamma from the unperturbed
    profile; v = 0.  Gravity g = -G M(<R) / R^2 (r, z) / R with
    M = 4 pi a^3 rho_c xi^2 |theta'| (the total mass outside the star).
    Reflecting at r = 0 and z = 0, transmissive outside.
    Returns (params, U, gravity[2, ny, nx])."""
    gamma = 1.0 + 1.0 / poly_n
    a = math.sqrt((poly_n + 1.0) * K * rho_c ** (1.0 / poly_n - 1.0) / (4.0 * math.pi * G))
    xi_t, th_t, ph_t, xi1 = lane_emden(poly_n, h)
    R = a * xi1
    L = extent * R
    p_floor = K * rho_floor ** gamma
    prm = make_params(n, n, 0.0, L, 0.0, L, [REFLECTING, TRANSMISSIVE, REFLECTING, TRANSMISSIVE],
                      gamma, cfl, geometry=CYLINDRICAL, rho_floor=rho_floor, p_floor=p_floor)
    r, z = centres(prm)
    Rr, Zz = np.meshgrid(r, z)
    Rad = np.sqrt(Rr * Rr + Zz * Zz)
    xi = Rad / a
    inside = xi < xi1
    theta = np.where(inside, np.interp(xi, xi_t, th_t), 0.0)
    dtheta = np.where(inside, np.interp(xi, xi_t, ph_t), ph_t[-1])
    rho_le = rho_c * _libm_pow(np.maximum(theta, 0.0), poly_n)
    rng = np.random.default_rng(seed)
    pert = 1.0 + noise * rng.uniform(-1.0, 1.0, (n, n))
    dense = rho_le > rho_floor
    rho = np.where(dense, rho_le * pert, rho_floor)
    p = K * _libm_pow(np.maximum(rho_le, rho_floor), gamma)
    xi_m = np.where(inside, xi, xi1)
    M = 4.0 * math.pi * a ** 3 * rho_c * xi_m ** 2 * np.abs(dtheta)
    gmag = -G * M / (Rad * Rad)
    grav = np.stack([gmag * Rr / Rad, gmag * Zz / Rad])
    U = state_from_primitive(rho, 0.0, 0.0, p, gamma)
    return prm, U, np.ascontiguousarray(grav)


def kh_sine_amplitudes(K=64, seed=5, std=1e-3):
    """a_k ~ N(0, std), k = 1..K."""
    return np.random.default_rng(seed).normal(0.0, std, K)


def kh_sine_params(n=1024, gamma=5.0 / 3.0, cfl=0.5):
    return make_params(n, n, 0.0, 1.0, 0.0, 1.0, [PERIODIC] * 4, gamma, cfl)


def kh_sine_state(a, params, xp=None):
    """Shear layer of :func:`kelvin_helmholtz` with v_y(x) = sum_k a_k sin(2 pi k x)
    (no noise).  ``a`` may be a numpy array or a torch tensor (then the state is
    a torch tensor on a's device, differentiable in a)."""
    nx, ny, gamma = params["nx"], params["ny"], params["gamma"]
    x, y = centres(params)
    inner = (np.abs(y - 0.5) < 0.25)[:, None] * np.ones((1, nx), dtype=bool)
    rho_np = np.where(inner, 2.0, 1.0)
    u_np = np.where(inner, 0.5, -0.5)
    k = np.arange(1, len(a) + 1)
    basis = _libm(math.sin, 2.0 * np.pi * np.outer(k, x))  # (K, nx)
    try:
        import torch
        is_torch = isinstance(a, torch.Tensor)
    except ImportError:  # pragma: no cover
        is_torch = False
    # v = a_1 B_1 + a_2 B_2 + ... summed in this order (elementwise products
    # and sums: the same values from numpy and from torch on any device)
    if not is_torch:
        an = np.asarray(a, dtype=np.float64)
        v = an[0] * basis[0]
        for m in range(1, len(an)):
            v = v + an[m] * basis[m]
        v = v[None, :] * np.ones((ny, 1))
        return state_from_primitive(rho_np, u_np, v, 2.5, gamma)
    import torch
    dev, dt = a.device, torch.float64
    rho = torch.as_tensor(rho_np, device=dev, dtype=dt)
    u = torch.as_tensor(u_np, device=dev, dtype=dt)
    B = torch.as_tensor(basis, device=dev, dtype=dt)
    ad = a.to(dt)
    vx = ad[0] * B[0]
    for m in range(1, ad.shape[0]):
        vx = vx + ad[m] * B[m]
    v = vx.unsqueeze(0).expand(ny, nx)
    E = 2.5 / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return torch.stack([rho, rho * u, rho * v, E]).contiguous()


# ------------------------------------------------------ smooth exact problems

def advection_1d(n, gamma=1.4, cfl=0.5, amp=0.2):
    """rho = 1 + amp sin(2 pi x), u = 1, p = 1 on periodic [0, 1] (1D limit).
    Exact solution at time t: rho(x - t)."""
    prm = make_params(n, 1, 0.0, 1.0, 0.0, 1.0, [PERIODIC, PERIODIC, TRANSMISSIVE, TRANSMISSIVE],
                      gamma, cfl)
    x, _ = centres(prm)
    rho = (1.0 + amp * np.sin(2.0 * np.pi * x))[None, :]
    return prm, state_from_primitive(rho, 1.0, 0.0, 1.0, gamma)


def advection_2d(n, gamma=1.4, cfl=0.5, amp=0.2):
    """rho = 1 + amp sin(2 pi (x + y)), u = v = 1, p = 1 on the periodic unit
    square.  Exact solution at time t: rho(x + y - 2 t)."""
    prm = make_params(n, n, 0.0, 1.0, 0.0, 1.0, [PERIODIC] * 4, gamma, cfl)
    x, y = centres(prm)
    X, Y = np.meshgrid(x, y)
    rho = 1.0 + amp * np.sin(2.0 * np.pi * (X + Y))
    return prm, state_from_primitive(rho, 1.0, 1.0, 1.0, gamma)


def homologous(n, a0, b0, geometry=CARTESIAN, rho0=1.0, p0=1.0, gamma=1.4, cfl=0.5, L=1.0):
    """Uniform rho, p with v = (a0 x, b0 y) on [0, L]^2 (x = r in cylindrical),
    reflecting at x = 0 and y = 0, transmissive outside.  Exact solution:
    a(t) = a0 / (1 + a0 t), b(t) = b0 / (1 + b0 t),
    rho(t) = rho0 / ((1 + a0 t)^m (1 + b0 t)) with m = 1 (Cartesian) or 2 (cylindrical),
    p = p0 (rho / rho0)^gamma."""
    prm = make_params(n, n, 0.0, L, 0.0, L, [REFLECTING, TRANSMISSIVE, REFLECTING, TRANSMISSIVE],
                      gamma, cfl, geometry=geometry)
    x, y = centres(prm)
    X, Y = np.meshgrid(x, y)
    return prm, state_from_primitive(rho0, a0 * X, b0 * Y, p0, gamma)


def gresho(n, gamma=1.4, cfl=0.5):
    """Gresho vortex of Sect. 5.2 on [-0.5, 0.5]^2 with free (transmissive) boundaries."""
    prm = make_params(n, n, -0.5, 0.5, -0.5, 0.5, [TRANSMISSIVE] * 4, gamma, cfl)
    x, y = centres(prm)
    X, Y = np.meshgrid(x, y)
    r = np.sqrt(X * X + Y * Y)
    vphi = np.where(r < 0.2, 5.0 * r, np.where(r < 0.4, 2.0 - 5.0 * r, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        p = np.where(r < 0.2, 5.0 + 12.5 * r * r,
                     np.where(r < 0.4, 9.0 + 4.0 * np.log(np.maximum(r, 1e-300) / 0.2)
                              + 12.5 * r * r - 20.0 * r, 3.0 + 4.0 * math.log(2.0)))
        s = np.where(r > 0, 1.0 / np.maximum(r, 1e-300), 0.0)
    u = -vphi * Y * s
    v = vphi * X * s
    return prm, state_from_primitive(1.0, u, v, p, gamma)


def blast(nx=512, ny=768, gamma=1.4, cfl=0.5):
    """Blast test of Sect. 5.2: [-0.5, 0.5] x [-0.75, 0.75], reflecting, rho = 1,
    p = 10 for r < 0.1 else 1."""
    prm = make_params(nx, ny, -0.5, 0.5, -0.75, 0.75, [REFLECTING] * 4, gamma, cfl)
    x, y = centres(prm)
    X, Y = np.meshgrid(x, y)
    p = np.where(X * X + Y * Y < 0.01, 10.0, 1.0)
    return prm, state_from_primitive(1.0, 0.0, 0.0, p, gamma)


def explosion(n=512, gamma=1.4, cfl=0.5):
    """Explosion test of Sect. 5.2: [0, 1.5]^2, reflecting at x = 0 and y = 0,
    free outside; (rho, p) = (1, 1) for r < 0.4 else (0.125, 0.1)."""
    prm = make_params(n, n, 0.0, 1.5, 0.0, 1.5, [REFLECTING, TRANSMISSIVE, REFLECTING, TRANSMISSIVE],
                      gamma, cfl)
    x, y = centres(prm)
    X, Y = np.meshgrid(x, y)
    inside = X * X + Y * Y < 0.16
    return prm, state_from_primitive(np.where(inside, 1.0, 0.125), 0.0, 0.0,
                                     np.where(inside, 1.0, 0.1), gamma)


def corners(params):
    """Corner coordinates (x of shape (nx+1,), y of shape (ny+1,))."""
    nx, ny = params["nx"], params["ny"]
    dx = (params["xhi"] - params["xlo"]) / nx
    dy = (params["yhi"] - params["ylo"]) / ny
    return params["xlo"] + np.arange(nx + 1) * dx, params["ylo"] + np.arange(ny + 1) * dy


def single_vortex(params, t=0.0, period=0.0):
    """Corner velocity (2, ny+1, nx+1) of the deforming single vortex on the unit
    square, u = -sin^2(pi x) sin(2 pi y), v = sin^2(pi y) sin(2 pi x), times
    cos(pi t / period) when a period is given."""
    x, y = corners(params)
    X, Y = np.meshgrid(x, y)
    f = math.cos(math.pi * t / period) if period > 0 else 1.0
    u = -f * np.sin(np.pi * X) ** 2 * np.sin(2 * np.pi * Y)
    v = f * np.sin(np.pi * Y) ** 2 * np.sin(2 * np.pi * X)
    return np.ascontiguousarray(np.stack([u, v]))


def flame_front(n=1024, seed=6, R0=0.2, modes=8, amp=0.03, slope=1.5, s_f=0.02):
    """Level-set workload on the (n+1)^2 corners of the unit square: ash (S > 0)
    inside a circle of radius R0 centred at (0.5, 0.75) whose radius carries
    seeded modes, R(theta) = R0 (1 + sum_k a_k cos(k theta + phi_k)),
    k = 2..modes+1, a_k ~ N(0, amp), phi_k ~ U(0, 2 pi); S = slope (R(theta) - r)
    (not a distance function unless slope = 1 and amp = 0); the single-vortex
    corner velocity; transmissive edges; laminar flame speed s_f.
    Returns (params, S, vel, s_f)."""
    prm = make_params(n, n, 0.0, 1.0, 0.0, 1.0, [TRANSMISSIVE] * 4, 1.4)
    x, y = corners(prm)
    X, Y = np.meshgrid(x, y)
    dxc, dyc = X - 0.5, Y - 0.75
    r = np.sqrt(dxc * dxc + dyc * dyc)
    th = np.arctan2(dyc, dxc)
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, amp, modes)
    ph = rng.uniform(0.0, 2 * np.pi, modes)
    Rt = np.ones_like(r)
    for k in range(modes):
        Rt = Rt + a[k] * np.cos((k + 2) * th + ph[k])
    S = slope * (R0 * Rt - r)
    return prm, np.ascontiguousarray(S), single_vortex(prm), float(s_f)
