"""The hydro step in plain PyTorch CPU float64 ops, for the reference gradient.

TEST INFRASTRUCTURE (see the package docstring): imported only by tests and
the benchmark's baseline leg.

The forward pass here is an independent second writing of the update that
``hydro_oracle.c`` performs (Sect. 2.1, Eq. euler2D; WENO5-JS of Jiang & Shu
1996 in its textbook form a_k = d_k / (eps + beta_k)^2, omega = a / sum a;
global Lax-Friedrichs split; SSP-RK3), vectorised with tensor slicing instead
of loops.  It agrees with the C oracle to rounding, not bit for bit.

Its purpose is the adjoint: with the time step dt and the LF speeds alpha of
each stage held at given (recorded) values, the step U -> U^{n+1} is a smooth
map, and ``torch.autograd`` applied to this forward yields the exact
vector-Jacobian product lambda -> J^T lambda of that map.  That is the
definition the hand-written device adjoint must reproduce.
"""
from __future__ import annotations

import torch

PERIODIC, TRANSMISSIVE, REFLECTING = 0, 1, 2
NG = 3


def _ghost_map(n, bc_lo, bc_hi):
    """Source index and normal-momentum sign for the padded axis of length n + 6."""
    src, sign = [], []
    for g in range(-NG, n + NG):
        s, f = g, 1.0
        if g < 0:
            if bc_lo == PERIODIC:
                s = g + n
            elif bc_lo == TRANSMISSIVE:
                s = 0
            else:
                s, f = -g - 1, -1.0
        elif g >= n:
            if bc_hi == PERIODIC:
                s = g - n
            elif bc_hi == TRANSMISSIVE:
                s = n - 1
            else:
                s, f = 2 * n - 1 - g, -1.0
        src.append(s)
        sign.append(f)
    return torch.tensor(src), torch.tensor(sign, dtype=torch.float64)


def _pad(V, axis, bc_lo, bc_hi, normal_comp):
    """Pad a (4, ny, nx) state along axis (2 = x, 1 = y) with three ghost layers."""
    n = V.shape[axis]
    src, sign = _ghost_map(n, bc_lo, bc_hi)
    P = V.index_select(axis, src)
    s = torch.ones(4, n + 2 * NG, dtype=V.dtype)
    s[normal_comp] = sign.to(V.dtype)
    s = s[:, None, :] if axis == 2 else s[:, :, None]
    return P * s


def _prims(V, gamma):
    rho, mx, my, E = V[0], V[1], V[2], V[3]
    u = mx / rho
    v = my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    c = torch.sqrt(gamma * p / rho)
    return rho, u, v, p, c


def _split(P, gamma, alpha, direction):
    rho, u, v, p, _ = _prims(P, gamma)
    mx, my, E = P[1], P[2], P[3]
    if direction == 0:
        F = torch.stack([mx, mx * u + p, my * u, (E + p) * u])
    else:
        F = torch.stack([my, mx * v, my * v + p, (E + p) * v])
    return 0.5 * (F + alpha * P), 0.5 * (F - alpha * P)


def weno5(v0, v1, v2, v3, v4, eps):
    """Textbook WENO5-JS value at the right face of v2 (elementwise)."""
    b0 = 13.0 / 12.0 * (v0 - 2 * v1 + v2) ** 2 + 0.25 * (v0 - 4 * v1 + 3 * v2) ** 2
    b1 = 13.0 / 12.0 * (v1 - 2 * v2 + v3) ** 2 + 0.25 * (v1 - v3) ** 2
    b2 = 13.0 / 12.0 * (v2 - 2 * v3 + v4) ** 2 + 0.25 * (3 * v2 - 4 * v3 + v4) ** 2
    a0 = 0.1 / (eps + b0) ** 2
    a1 = 0.6 / (eps + b1) ** 2
    a2 = 0.3 / (eps + b2) ** 2
    s = a0 + a1 + a2
    q0 = (2 * v0 - 7 * v1 + 11 * v2) / 6.0
    q1 = (-v1 + 5 * v2 + 2 * v3) / 6.0
    q2 = (2 * v2 + 5 * v3 - v4) / 6.0
    return (a0 * q0 + a1 * q1 + a2 * q2) / s


def _face_flux(fp, fm, axis, n, eps):
    """F-hat at the n + 1 faces along a padded axis (length n + 6)."""
    def sl(k):  # padded points k .. k + n (n + 1 of them); face f has left cell f - 1 -> padded f + 2
        return fp.narrow(axis, k, n + 1), fm.narrow(axis, k, n + 1)
    # face f: W+(fp[f..f+4] padded, i.e. cells f-3..f+1) + W-(fm[f+5..f+1] padded)
    p0, m0 = sl(0)
    p1, m1 = sl(1)
    p2, m2 = sl(2)
    p3, m3 = sl(3)
    p4, m4 = sl(4)
    _, m5 = sl(5)
    return weno5(p0, p1, p2, p3, p4, eps) + weno5(m5, m4, m3, m2, m1, eps)


def rhs(params, gravity, V, ax, ay):
    """L(V) = S(V) - (dF/dx + dG/dy) for given LF speeds (ax, ay)."""
    nx, ny = params["nx"], params["ny"]
    gamma, eps = params["gamma"], params.get("eps", 1e-6)
    bc = params["bc"]
    dx = (params["xhi"] - params["xlo"]) / nx
    dy = (params["yhi"] - params["ylo"]) / ny
    Px = _pad(V, 2, bc[0], bc[1], 1)
    fp, fm = _split(Px, gamma, ax, 0)
    Fh = _face_flux(fp, fm, 2, nx, eps)
    D = (Fh[:, :, 1:] - Fh[:, :, :-1]) / dx
    if ny > 1:
        Py = _pad(V, 1, bc[2], bc[3], 2)
        gp, gm = _split(Py, gamma, ay, 1)
        Gh = _face_flux(gp, gm, 1, ny, eps)
        D = D + (Gh[:, 1:, :] - Gh[:, :-1, :]) / dy
    rho, u, v, p, _ = _prims(V, gamma)
    if gravity is None:
        gx = torch.full_like(rho, params.get("gx", 0.0))
        gy = torch.full_like(rho, params.get("gy", 0.0))
    else:
        gx, gy = gravity[0], gravity[1]
    S = torch.stack([torch.zeros_like(rho), rho * gx, rho * gy, V[1] * gx + V[2] * gy])
    if params.get("geometry", 0) == 1:
        r = (params["xlo"] + (torch.arange(nx, dtype=torch.float64) + 0.5) * dx).to(V.dtype)
        geo = torch.stack([V[1], V[1] * u, V[2] * u, (V[3] + p) * u]) / r
        S = S - geo
    return S - D


def step(params, gravity, U, dt, alpha):
    """One SSP-RK3 step with LF speeds alpha[s] = (ax, ay) for stages s = 0, 1, 2."""
    U1 = U + dt * rhs(params, gravity, U, *alpha[0])
    U2 = 0.75 * U + 0.25 * (U1 + dt * rhs(params, gravity, U1, *alpha[1]))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * rhs(params, gravity, U2, *alpha[2]))


def _as_t(a, dtype=torch.float64):
    return torch.as_tensor(a, dtype=torch.float64).to(dtype)


def step_np(params, gravity, U, dt, alpha):
    """Numpy in, numpy out forward step (frozen alpha)."""
    g = None if gravity is None else _as_t(gravity)
    with torch.no_grad():
        return step(params, g, _as_t(U), float(dt), [tuple(map(float, a)) for a in alpha]).numpy()


def vjp(params, gravity, U, dt, alpha, lam, dtype=torch.float64):
    """J^T lam for one step at state U (dt, alpha frozen).  Numpy in/out.
    dtype=torch.float32 evaluates the same step and its autograd entirely in
    single precision (inputs rounded to it, result returned as float64): the
    error that precision alone brings to the adjoint."""
    g = None if gravity is None else _as_t(gravity, dtype)
    x = _as_t(U, dtype).clone().requires_grad_(True)
    y = step(params, g, x, float(dt), [tuple(map(float, a)) for a in alpha])
    (gx,) = torch.autograd.grad(y, x, _as_t(lam, dtype))
    return gx.double().numpy()


def vjp_steps(params, gravity, U, dts, alphas, lam):
    """J^T lam through several steps (recorded dts, alphas), by autograd."""
    g = None if gravity is None else _as_t(gravity)
    x = _as_t(U).clone().requires_grad_(True)
    y = x
    for dt, al in zip(dts, alphas):
        y = step(params, g, y, float(dt), [tuple(map(float, a)) for a in al])
    (gx,) = torch.autograd.grad(y, x, _as_t(lam))
    return gx.numpy()
