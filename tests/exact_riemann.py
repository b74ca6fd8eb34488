"""Exact solution of the Riemann problem for the 1D Euler equations (ideal gas).

Used to pin the oracle on the shock-tube problems of Sect. 5.1, whose
reference solutions the paper says are computed by exact Riemann solvers.

Method: the star-region pressure p* is the root of
    f(p) = f_L(p) + f_R(p) + (u_R - u_L),
where f_K is the velocity jump across the K wave: the shock branch
(p - p_K) sqrt(A_K / (p + B_K)) with A_K = 2 / ((gamma+1) rho_K),
B_K = (gamma-1)/(gamma+1) p_K when p > p_K (Rankine-Hugoniot), and the
rarefaction branch 2 c_K / (gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1)
otherwise (isentropic, Riemann invariant).  f is monotone and concave, so
Newton's method from a positive start converges.  u* = (u_L + u_R)/2 +
(f_R(p*) - f_L(p*))/2.  The self-similar solution is sampled at x/t.
"""
from __future__ import annotations

import math

import numpy as np


class RiemannSolution:
    def __init__(self, rho_l, u_l, p_l, rho_r, u_r, p_r, gamma=1.4):
        self.g = float(gamma)
        self.L = (float(rho_l), float(u_l), float(p_l))
        self.R = (float(rho_r), float(u_r), float(p_r))
        g = self.g
        self.cl = math.sqrt(g * p_l / rho_l)
        self.cr = math.sqrt(g * p_r / rho_r)
        if 2.0 * (self.cl + self.cr) / (g - 1.0) <= (u_r - u_l):
            raise ValueError("vacuum is generated; not supported")
        self.p_star, self.u_star = self._star()

    def _fk(self, p, rho_k, p_k, c_k):
        g = self.g
        if p > p_k:
            A = 2.0 / ((g + 1.0) * rho_k)
            B = (g - 1.0) / (g + 1.0) * p_k
            f = (p - p_k) * math.sqrt(A / (p + B))
            df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - p_k) / (B + p))
        else:
            e = (g - 1.0) / (2.0 * g)
            f = 2.0 * c_k / (g - 1.0) * ((p / p_k) ** e - 1.0)
            df = (p / p_k) ** (-(g + 1.0) / (2.0 * g)) / (rho_k * c_k)
        return f, df

    def _star(self):
        (rl, ul, pl), (rr, ur, pr) = self.L, self.R
        g = self.g
        # two-rarefaction estimate as the start (always positive)
        e = (g - 1.0) / (2.0 * g)
        p = ((self.cl + self.cr - 0.5 * (g - 1.0) * (ur - ul))
             / (self.cl / pl ** e + self.cr / pr ** e)) ** (1.0 / e)
        for _ in range(200):
            fl, dfl = self._fk(p, rl, pl, self.cl)
            fr, dfr = self._fk(p, rr, pr, self.cr)
            p_new = p - (fl + fr + ur - ul) / (dfl + dfr)
            if p_new <= 0.0:
                p_new = 0.5 * p
            if abs(p_new - p) <= 1e-15 * (p_new + p):
                p = p_new
                break
            p = p_new
        fl, _ = self._fk(p, rl, pl, self.cl)
        fr, _ = self._fk(p, rr, pr, self.cr)
        return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)

    # --- wave structure -------------------------------------------------
    def star_density(self, side):
        g = self.g
        rk, uk, pk = self.L if side == "L" else self.R
        ps = self.p_star
        if ps > pk:
            q = ps / pk
            return rk * (q + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * q + 1.0)
        return rk * (ps / pk) ** (1.0 / g)

    def shock_speed(self, side):
        g = self.g
        rk, uk, pk = self.L if side == "L" else self.R
        ck = self.cl if side == "L" else self.cr
        q = self.p_star / pk
        w = ck * math.sqrt((g + 1.0) / (2.0 * g) * q + (g - 1.0) / (2.0 * g))
        return uk - w if side == "L" else uk + w

    def sample(self, s):
        """(rho, u, p) at similarity coordinate s = (x - x0) / t (array ok)."""
        s = np.asarray(s, dtype=np.float64)
        out = np.empty((3,) + s.shape)
        flat = [self._sample1(float(v)) for v in s.ravel()]
        arr = np.array(flat).T.reshape((3,) + s.shape)
        out[:] = arr
        return out

    def _sample1(self, s):
        g = self.g
        (rl, ul, pl), (rr, ur, pr) = self.L, self.R
        ps, us = self.p_star, self.u_star
        if s <= us:  # left of the contact
            if ps > pl:
                return (rl, ul, pl) if s < self.shock_speed("L") else (self.star_density("L"), us, ps)
            c_star = self.cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
            head, tail = ul - self.cl, us - c_star
            if s <= head:
                return (rl, ul, pl)
            if s >= tail:
                return (self.star_density("L"), us, ps)
            u = 2.0 / (g + 1.0) * (self.cl + 0.5 * (g - 1.0) * ul + s)
            c = 2.0 / (g + 1.0) * (self.cl + 0.5 * (g - 1.0) * (ul - s))
            rho = rl * (c / self.cl) ** (2.0 / (g - 1.0))
            return (rho, u, pl * (c / self.cl) ** (2.0 * g / (g - 1.0)))
        if ps > pr:
            return (rr, ur, pr) if s > self.shock_speed("R") else (self.star_density("R"), us, ps)
        c_star = self.cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
        head, tail = ur + self.cr, us + c_star
        if s >= head:
            return (rr, ur, pr)
        if s <= tail:
            return (self.star_density("R"), us, ps)
        u = 2.0 / (g + 1.0) * (-self.cr + 0.5 * (g - 1.0) * ur + s)
        c = 2.0 / (g + 1.0) * (self.cr - 0.5 * (g - 1.0) * (ur - s))
        rho = rr * (c / self.cr) ** (2.0 / (g - 1.0))
        return (rho, u, pr * (c / self.cr) ** (2.0 * g / (g - 1.0)))


def cell_average(sol, x_edges, x0, t, sub=64):
    """Cell averages of (rho, u, p) over cells with the given edges (for L1 norms
    against point values, the point value at the centre is used instead by the
    tests; this helper is for diagnostics)."""
    out = []
    for a, b in zip(x_edges[:-1], x_edges[1:]):
        xs = a + (np.arange(sub) + 0.5) * (b - a) / sub
        out.append(sol.sample((xs - x0) / t).mean(axis=1))
    return np.array(out).T
