"""Pins of the level-set oracle (Sect. 2.3: advection of the corner field by
dS/dt = -(v + v_flame) . grad S with the WENO scheme, then re-distancing by
front points from linear interpolation, the nearest distance and the tanh
blend with d0 = 3 D and width D/3).

Against facts fixed independently of the oracle's code:
* front points of a hand-worked 3 x 2 corner field;
* a straight front: the nearest distance is the distance to the line, nodes
  on the front keep their value, the blend gives the old value within one
  spacing (H(D) = 1 - 6e-6), the midpoint of old value and distance at
  d = 3 D (H(3D) = 1/(1 + tanh 9)), the distance beyond 6 D (H < 2e-8);
* a circle: far from the front the new value is the distance to the circle
  within the second-order error of piecewise-linear front placement;
* advection of linear fields is exact (WENO5 reproduces constant slopes):
  translation by the velocity and, with a flame speed, growth of the burnt
  side at s_f (this fixes the sign of the flame term);
* fifth-order convergence of smooth periodic translation;
* the reflecting corner boundary equals the mirror-symmetric periodic problem
  on the doubled domain;
* a circular flame with no flow grows at s_f.
"""
import math

import numpy as np
import pytest

from paper_1507_08549_amd import inputs

P, T, R = inputs.PERIODIC, inputs.TRANSMISSIVE, inputs.REFLECTING


def _prm(nx, ny, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0, bc=(T, T, T, T)):
    return inputs.make_params(nx, ny, xlo, xhi, ylo, yhi, list(bc), 1.4)


def test_front_points_by_hand(oracle_mod):
    # corners (x, y) = (i, j), i = 0..2, j = 0..1
    ls = oracle_mod.LevelSet(_prm(2, 1, 0.0, 2.0, 0.0, 1.0))
    S = np.array([[-1.0, 3.0, 3.0],
                  [1.0, 1.0, -1.0]])
    got = {tuple(p) for p in ls.front(S)}
    # row 0: (-1, 3) at x = 1/4; row 1: (1, -1) at x = 1.5;
    # column 0: (-1, 1) at y = 1/2; column 2: (3, -1) at y = 3/4
    assert got == {(0.25, 0.0), (1.5, 1.0), (0.0, 0.5), (2.0, 0.75)}
    # a corner at zero is a front point; its edges give none
    S2 = np.array([[0.0, 2.0, 3.0], [1.0, 1.0, 1.0]])
    assert {tuple(p) for p in ls.front(S2)} == {(0.0, 0.0)}


def test_no_front_leaves_the_field(oracle_mod):
    ls = oracle_mod.LevelSet(_prm(8, 8))
    S = 1.0 + np.random.default_rng(0).uniform(0, 1, (9, 9))
    Sn, d, n = ls.redistance(S)
    assert n == 0 and d is None and np.array_equal(Sn, S)


def test_straight_front_blend(oracle_mod):
    n = 64
    D = 1.0 / n
    prm = _prm(n, n)
    ls = oracle_mod.LevelSet(prm)
    x, y = inputs.corners(prm)
    X, _ = np.meshgrid(x, y)
    x0 = 0.5                       # a corner column: exact distances k D
    c = 2.5                        # a slope that is not 1
    S = c * (x0 - X)               # ash on the left
    Sn, d, npts = ls.redistance(S)
    assert npts == n + 1
    dist = np.abs(X - x0)
    assert np.array_equal(d, dist)
    k = np.rint(dist / D).astype(int)
    sd = np.sign(S) * dist
    assert np.array_equal(Sn[k == 0], S[k == 0])
    near = k == 1
    assert np.allclose(Sn[near], S[near], rtol=1e-5, atol=0)
    mid = k == 3
    assert np.allclose(Sn[mid], 0.5 * (S[mid] + sd[mid]), rtol=1e-7, atol=0)
    far = k >= 6
    assert np.allclose(Sn[far], sd[far], rtol=2e-8 * c, atol=0)
    # monotone transition between the old value and the distance
    w = (Sn - sd) / (S - sd + (k == 0))
    row = w[0, n // 2 + 1:]
    assert np.all(np.diff(row) <= 0) and row[0] > 0.9999 and row[-1] < 1e-12


def test_circle_far_field_is_the_distance(oracle_mod):
    n = 128
    D = 1.0 / n
    prm = _prm(n, n)
    ls = oracle_mod.LevelSet(prm)
    x, y = inputs.corners(prm)
    X, Y = np.meshgrid(x, y)
    r = np.sqrt((X - 0.43) ** 2 + (Y - 0.52) ** 2)
    R0 = 0.27
    S = 1.7 * (R0 - r) + 0.2 * (R0 - r) ** 2
    Sn, d, npts = ls.redistance(S)
    # linear interpolation places the front points on the circle to O(D^2 / R0)
    pts = ls.front(S)
    pr = np.sqrt((pts[:, 0] - 0.43) ** 2 + (pts[:, 1] - 0.52) ** 2)
    assert np.abs(pr - R0).max() < 0.01 * D
    # the nearest of points spaced at most sqrt(2) D apart along the circle is
    # farther than the circle by at most (r / R0) s^2 / (8 rho) at distance rho
    exact = np.abs(r - R0)
    far = (exact > 6.5 * D) & (r > 0.05)
    bound = np.maximum(r, R0) / R0 * (2 * D * D) / (8 * exact) + 0.01 * D
    err = Sn - np.sign(R0 - r) * exact
    assert np.all(np.abs(err[far]) <= bound[far]), (np.abs(err[far]) / bound[far]).max()
    # and never nearer than the circle (beyond the placement error)
    assert np.all(np.abs(Sn[far]) >= exact[far] - 0.01 * D)
    # the number of front points is about the number of edges the circle crosses
    assert 0.9 < npts / (8 * R0 / D) < 1.5


def test_linear_field_translates_exactly(oracle_mod):
    n = 24
    prm = _prm(n, n)
    ls = oracle_mod.LevelSet(prm)
    x, y = inputs.corners(prm)
    X, Y = np.meshgrid(x, y)
    a, b = 0.6, -0.8
    S = a * X + b * Y + 0.1
    vel = np.stack([np.full_like(X, 0.3), np.full_like(X, -0.7)])
    dt = 0.01
    S1 = ls.step(S, vel, 0.0, dt)
    np.testing.assert_allclose(S1, S - (a * 0.3 + b * -0.7) * dt, rtol=0, atol=1e-14)
    # |grad S| = 1 and a flame speed: the burnt side (S > 0) grows at s_f
    s_f = 0.25
    S2 = ls.step(S, vel, s_f, dt)
    np.testing.assert_allclose(S2, S + (s_f - (a * 0.3 + b * -0.7)) * dt, rtol=0, atol=1e-14)
    # speeds: max |u| + s_f, max |v| + s_f
    assert np.array_equal(ls.alpha(vel, s_f), [0.3 + s_f, 0.7 + s_f])


def _translate(oracle_mod, n, t_end=0.25):
    prm = _prm(n, n, bc=(P, P, P, P))
    ls = oracle_mod.LevelSet(prm)
    x, y = inputs.corners(prm)
    X, Y = np.meshgrid(x, y)
    f = lambda X, Y: np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) / (2 * np.pi)
    S = f(X, Y)
    vel = np.stack([np.full_like(X, 1.0), np.full_like(X, 0.5)])
    dt = 0.3 * (1.0 / n) ** (5.0 / 3.0)
    nst = int(np.ceil(t_end / dt))
    dt = t_end / nst
    for _ in range(nst):
        S = ls.step(S, vel, 0.0, dt)
    assert np.array_equal(S[:, -1], S[:, 0]) and np.array_equal(S[-1], S[0])
    return np.abs(S - f(X - t_end, Y - 0.5 * t_end)).mean()


def test_fifth_order_translation(oracle_mod):
    errs = [_translate(oracle_mod, n) for n in (16, 32, 64)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > 4.5, (errs, orders)


def test_reflecting_equals_mirrored_periodic(oracle_mod):
    n = 32
    half = _prm(n, n, 0.0, 1.0, 0.0, 1.0, bc=(R, R, T, T))  # the seam x = +-1 is a mirror too
    full = _prm(2 * n, n, -1.0, 1.0, 0.0, 1.0, bc=(P, P, T, T))
    xf, yf = inputs.corners(full)
    X, Y = np.meshgrid(xf, yf)
    S = 0.3 - np.sqrt((np.abs(X) - 0.5) ** 2 + (Y - 0.4) ** 2) + 0.1 * np.cos(np.pi * X)
    vel = np.stack([np.sin(np.pi * X) * Y, np.cos(np.pi * X) * (1 - Y)])
    a = oracle_mod.LevelSet(full).alpha(vel, 0.1)
    Sf, Sh = S.copy(), np.ascontiguousarray(S[:, n:])
    vh = np.ascontiguousarray(vel[:, :, n:])
    lf, lh = oracle_mod.LevelSet(full), oracle_mod.LevelSet(half)
    assert np.array_equal(lh.alpha(vh, 0.1), a)
    for _ in range(5):
        Sf = lf.step(Sf, vel, 0.1, 0.004)
        Sh = lh.step(Sh, vh, 0.1, 0.004)
    np.testing.assert_allclose(Sh, Sf[:, n:], rtol=0, atol=1e-14)


def test_circular_flame_grows_at_the_flame_speed(oracle_mod):
    n = 128
    prm = _prm(n, n)
    ls = oracle_mod.LevelSet(prm)
    x, y = inputs.corners(prm)
    X, Y = np.meshgrid(x, y)
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2)
    S = 0.2 - r
    vel = np.zeros((2,) + S.shape)
    s_f, dt, nst = 0.5, 0.002, 100
    for k in range(nst):
        S = ls.step(S, vel, s_f, dt)
        if k % 10 == 9:
            S, _, _ = ls.redistance(S)
    # radius of the zero contour along the four axis directions
    t = s_f * dt * nst
    for row in (S[n // 2, n // 2:], S[n // 2, n // 2::-1], S[n // 2:, n // 2], S[n // 2::-1, n // 2]):
        k = np.nonzero(row < 0)[0][0]
        rad = (k - 1 + row[k - 1] / (row[k - 1] - row[k])) / n
        assert abs(rad - (0.2 + t)) < 0.05 / n, (rad, 0.2 + t)


def test_corner_velocity(oracle_mod):
    """Linear velocity fields are reproduced exactly at interior corners (the
    mean of four cells about their shared corner); reflecting walls give zero
    normal velocity on the wall; periodic corners match their images."""
    n = 12
    prm = _prm(n, n - 2, bc=(R, T, P, P))
    ls = oracle_mod.LevelSet(prm)
    xc, yc = inputs.centres(prm)
    Xc, Yc = np.meshgrid(xc, yc)
    rho = 1.0 + 0.5 * Xc * Yc
    u, v = 0.25 + 0.5 * Xc - Yc, -0.5 + 0.75 * Xc
    U = inputs.state_from_primitive(rho, u, v, np.ones_like(rho), 1.4)
    vel = ls.corner_velocity(U)
    x, y = inputs.corners(prm)
    X, Y = np.meshgrid(x, y)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(vel[0][inner], (0.25 + 0.5 * X - Y)[inner], rtol=0, atol=1e-15)
    np.testing.assert_allclose(vel[1][inner], (-0.5 + 0.75 * X)[inner], rtol=0, atol=1e-15)
    assert np.all(vel[0][:, 0] == 0.0)                      # reflecting x-low wall
    np.testing.assert_allclose(vel[0][:, -1][1:-1], (0.5 * (u[:-1, -1] + u[1:, -1]))[:], atol=1e-15)
    assert np.array_equal(vel[:, 0, :], vel[:, -1, :])    # periodic in y
