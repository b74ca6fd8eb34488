"""Pins of the oracle's potential solver (Sect. 2.1: Poisson equation in
(r, z) by over-relaxed Gauss-Seidel, reflecting axis and plane, Roche outer
boundary) against closed forms: the n = 1 polytrope (density sin(xi)/xi,
potential -4 pi G a^2 rho_c (sin(xi)/xi + 1) inside, -GM/R outside) and the
uniform sphere (-2 pi G rho (a^2 - R^2/3) inside)."""
import math

import numpy as np
import pytest


def _grid(n, L):
    r = (np.arange(n) + 0.5) * L / n
    R, Z = np.meshgrid(r, r)
    return R, Z, np.sqrt(R * R + Z * Z)


def _poly1(n, L=1.25, G=1.0, rhoc=1.0):
    a = 1.0 / math.pi  # surface at R = 1
    R, Z, Rs = _grid(n, L)
    xi = Rs / a
    rho = np.where(xi < math.pi, rhoc * np.sinc(xi / math.pi), 0.0)
    M = 4 * math.pi ** 2 * a ** 3 * rhoc
    exact = np.where(xi < math.pi, -4 * math.pi * G * a * a * rhoc * (np.sinc(xi / math.pi) + 1), -G * M / Rs)
    menc = np.where(xi < math.pi, 4 * math.pi * a ** 3 * rhoc * (np.sin(xi) - xi * np.cos(xi)), M)
    g = -G * menc / Rs ** 2
    return rho, M, exact, np.stack([g * R / Rs, g * Z / Rs])


def test_second_order_on_the_n1_polytrope(oracle_mod):
    errs, gerrs = [], []
    for n in (32, 64, 128):
        rho, M, exact, gex = _poly1(n)
        phi, it, ch = oracle_mod.poisson(rho, 1.25, 1.25, 1.0, M,
                                         omega=2 / (1 + math.sin(math.pi / n)), tol=1e-12)
        assert ch < 1e-12 and it < 5000
        errs.append(np.abs(phi - exact).max() / np.abs(exact).max())
        g = oracle_mod.gravity_from_potential(phi, 1.25, 1.25, 1.0, M)
        gerrs.append(np.abs(g - gex).max() / np.abs(gex).max())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    gorder = np.log2(np.array(gerrs[:-1]) / np.array(gerrs[1:]))
    assert errs[0] < 1e-3 and np.all(order > 1.8), (errs, order)
    assert np.all(gorder > 1.5), (gerrs, gorder)


def test_uniform_sphere(oracle_mod):
    """A density jump: the staircase surface limits the error to first order."""
    errs = []
    for n in (32, 64, 128):
        R, Z, Rs = _grid(n, 1.0)
        rho = np.where(Rs < 0.5, 1.0, 0.0)
        M = 4 / 3 * math.pi * 0.125
        phi, _, _ = oracle_mod.poisson(rho, 1.0, 1.0, 1.0, M, omega=2 / (1 + math.sin(math.pi / n)), tol=1e-12)
        exact = np.where(Rs < 0.5, -2 * math.pi * (0.25 - Rs * Rs / 3), -M / Rs)
        errs.append(np.abs(phi - exact).max() / np.abs(exact).max())
    assert errs[0] < 0.02 and errs[-1] < errs[0] / 3, errs


def test_converged_solution_does_not_depend_on_omega(oracle_mod):
    rho, M, _, _ = _poly1(48)
    a, _, _ = oracle_mod.poisson(rho, 1.25, 1.25, 1.0, M, omega=1.2, tol=1e-13, max_iter=200000)
    b, _, _ = oracle_mod.poisson(rho, 1.25, 1.25, 1.0, M, omega=1.9, tol=1e-13, max_iter=200000)
    assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()


def test_discrete_equation_holds_at_convergence(oracle_mod):
    """Residual of the five-point equation (flux form in r, mirror at z = 0,
    Roche ghosts) after convergence, evaluated here independently."""
    n, L, G = 40, 1.25, 1.0
    rho, M, _, _ = _poly1(n, L, G)
    phi, _, _ = oracle_mod.poisson(rho, L, L, G, M, omega=1.8, tol=1e-14, max_iter=200000)
    d = L / n
    r = (np.arange(n) + 0.5) * d
    z = r
    roche = lambda rr, zz: -G * M / np.sqrt(rr * rr + zz * zz)
    P = np.zeros((n + 2, n + 1))  # rows j = -1..n, columns i = 0..n
    P[1:n + 1, :n] = phi
    P[1:n + 1, n] = roche(r[-1] + d, z)
    P[n + 1, :n] = roche(r, z[-1] + d)
    P[0, :n] = phi[0]  # mirror at z = 0
    i = np.arange(n)
    rp, rm = (i + 1) * d, i * d
    lap_r = (rp * (P[1:n + 1, 1:] - phi) - rm * (phi - np.concatenate([phi[:, :1], phi[:, :-1]], axis=1))) / (r * d * d)
    lap_z = (P[2:, :n] - 2 * phi + P[:n, :n]) / (d * d)
    res = lap_r + lap_z - 4 * math.pi * G * rho
    assert np.abs(res).max() <= 1e-7 * (4 * math.pi * G * rho.max())
