"""Pins of the oracle's reductions by hand-worked values and closed forms:

* the global Lax-Friedrichs speeds of Sect. 2.1, alpha_x = max(|u| + c) and
  alpha_y = max(|v| + c) over the interior, and the CFL speed of Sect. 5.3,
  s_max = max(c + |u| + |v|), on a grid whose three maxima sit in three
  different cells (a swapped pair, a dropped |v| or a missing 1/rho in c moves
  at least one of them);
* the CFL step dt = c_cfl min(dx, dy) / s_max (dx alone in the 1D limit) and
  its clamp to t_end;
* the conserved totals behind the Delta M / M, Delta E / E diagnostics of the
  paper's Gresho table (Sect. 5.2): uniform states against the closed-form
  volumes (rho times the area, or rho pi (r_hi^2 - r_lo^2) Z in (r, z): the
  midpoint rule is exact for the linear integrand 2 pi r), random states
  against math.fsum, and a cancellation that only compensated summation
  survives;
* the same results for any number of oracle threads, bit for bit.
"""
import math

import numpy as np
import pytest

from paper_1507_08549_amd import inputs

P, T, R = inputs.PERIODIC, inputs.TRANSMISSIVE, inputs.REFLECTING
GAMMA = 1.4


def _cell(rho, u, v, c):
    """Conserved values of a cell with density rho, velocity (u, v), sound speed c."""
    p = c * c * rho / GAMMA
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def _speed_grid(nx=5, ny=4, ylen=2.0, xlen=1.0):
    """Background at rest with c = 0.5; four cells set by hand:
    A (c = 1, u = 0.3, v = -0.4):      |u|+c 1.3,  |v|+c 1.4,  c+|u|+|v| 1.7
    E (rho = 4, c = 0.5, u = -1.05):   |u|+c 1.55 (alpha_x)
    C (c = 0.5, v = -1.1):             |v|+c 1.6  (alpha_y)
    D (c = 0.5, u = 0.6, v = 0.65):    c+|u|+|v| 1.75 (s_max)."""
    prm = inputs.make_params(nx, ny, 0.0, xlen, 0.0, ylen, [T] * 4, GAMMA, cfl=0.6)
    U = np.empty((4, ny, nx))
    U[:] = _cell(1.0, 0.0, 0.0, 0.5)[:, None, None]
    U[:, 0, 1] = _cell(1.0, 0.3, -0.4, 1.0)
    U[:, 1, 3] = _cell(4.0, -1.05, 0.0, 0.5)
    U[:, 2, 0] = _cell(1.0, 0.0, -1.1, 0.5)
    U[:, 3, 4] = _cell(1.0, 0.6, 0.65, 0.5)
    return prm, U


def test_lf_and_cfl_speeds_by_hand(oracle_mod):
    prm, U = _speed_grid()
    a = oracle_mod.Oracle(prm).alpha(U)
    np.testing.assert_allclose(a, [1.55, 1.6, 1.75], rtol=4e-16 * 8, atol=0)


def test_speeds_of_a_single_cell(oracle_mod):
    # rho = 1, p = 1 / gamma: c = 1; u = 0.3, v = -0.4
    prm = inputs.make_params(3, 3, 0.0, 1.0, 0.0, 1.0, [P] * 4, GAMMA)
    U = np.repeat(np.repeat(_cell(1.0, 0.3, -0.4, 1.0)[:, None, None], 3, 1), 3, 2)
    np.testing.assert_allclose(oracle_mod.Oracle(prm).alpha(U), [1.3, 1.4, 1.7], rtol=4e-15, atol=0)


def test_speeds_ignore_nothing_in_1d(oracle_mod):
    # 1D limit: a transverse momentum still counts in |v| + c and s_max
    prm = inputs.make_params(4, 1, 0.0, 1.0, 0.0, 1.0, [T] * 4, GAMMA)
    U = np.repeat(_cell(1.0, -0.2, 0.5, 1.0)[:, None, None], 4, 2)
    np.testing.assert_allclose(oracle_mod.Oracle(prm).alpha(U), [1.2, 1.5, 1.7], rtol=4e-15, atol=0)


@pytest.mark.parametrize("xlen, ylen, delta", [(1.0, 2.0, 0.2), (1.0, 0.4, 0.1)])
def test_cfl_step_uses_the_smaller_spacing(oracle_mod, xlen, ylen, delta):
    # 5 x 4 cells: dx = xlen / 5, dy = ylen / 4
    prm, U = _speed_grid(xlen=xlen, ylen=ylen)
    dt = oracle_mod.Oracle(prm).cfl(U)
    assert dt == pytest.approx(0.6 * delta / 1.75, rel=1e-15)


def test_cfl_step_in_1d_uses_dx(oracle_mod):
    # dy = 0.01 < dx = 0.125 must not enter the 1D limit
    prm = inputs.make_params(8, 1, 0.0, 1.0, 0.0, 0.01, [T] * 4, GAMMA, cfl=0.6)
    U = np.repeat(_cell(1.0, 0.3, 0.0, 1.0)[:, None, None], 8, 2)
    assert oracle_mod.Oracle(prm).cfl(U) == pytest.approx(0.6 * 0.125 / 1.3, rel=1e-15)


def test_run_clamps_the_last_step_to_t_end(oracle_mod):
    prm, U0 = inputs.sod(100)
    o = oracle_mod.Oracle(prm)
    U, t, dts, _ = o.run(U0, 10000, t_end=0.05)
    assert t == 0.05 and len(dts) >= 2
    # every step but the last is the CFL step of its start state; the last ends at t_end
    W, tt = U0.copy(), 0.0
    for k, dt in enumerate(dts):
        full = o.cfl(W)
        if k < len(dts) - 1:
            assert dt == full
        else:
            assert dt == 0.05 - tt and dt <= full
        W, _ = o.step(W, dt)
        tt = tt + dt
    assert np.array_equal(W, U)


@pytest.mark.parametrize("geometry, xlo", [(inputs.CARTESIAN, 0.5), (inputs.CYLINDRICAL, 0.0),
                                            (inputs.CYLINDRICAL, 0.3)])
def test_totals_of_uniform_states(oracle_mod, geometry, xlo):
    nx, ny, xhi, ylo, yhi = 37, 23, 2.0, -1.0, 0.5
    prm = inputs.make_params(nx, ny, xlo, xhi, ylo, yhi, [T] * 4, GAMMA, geometry=geometry)
    vals = np.array([1.7, -0.3, 0.25, 4.1])
    U = np.ascontiguousarray(np.broadcast_to(vals[:, None, None], (4, ny, nx)))
    if geometry == inputs.CARTESIAN:
        vol = (xhi - xlo) * (yhi - ylo)
    else:
        vol = math.pi * (xhi * xhi - xlo * xlo) * (yhi - ylo)
    np.testing.assert_allclose(oracle_mod.Oracle(prm).sums(U), vals * vol, rtol=1e-14, atol=0)


@pytest.mark.parametrize("geometry", [inputs.CARTESIAN, inputs.CYLINDRICAL])
def test_totals_of_random_states_match_fsum(oracle_mod, geometry):
    nx, ny = 29, 17
    prm = inputs.make_params(nx, ny, 0.0, 1.3, 0.0, 0.7, [T] * 4, GAMMA, geometry=geometry)
    rng = np.random.default_rng(11)
    U = rng.standard_normal((4, ny, nx)) * np.array([1.0, 10.0, 1e-3, 1e4])[:, None, None]
    dx, dy = 1.3 / nx, 0.7 / ny
    r = (np.arange(nx) + 0.5) * dx
    w = np.full(nx, dx * dy) if geometry == inputs.CARTESIAN else 2.0 * math.pi * r * (dx * dy)
    got = oracle_mod.Oracle(prm).sums(U)
    for c in range(4):
        terms = (U[c] * w[None, :]).ravel()
        want = math.fsum(terms)
        # per-term rounding of the volume factor (a few ulp) bounds the difference
        assert abs(got[c] - want) <= 1e-15 * math.fsum(np.abs(terms)), (c, got[c], want)


def test_totals_are_compensated(oracle_mod):
    # unit cells; m_x = (1e16, 1, -1e16) sums to 1 exactly, plain summation gives 0
    prm = inputs.make_params(3, 1, 0.0, 3.0, 0.0, 1.0, [T] * 4, GAMMA)
    U = np.zeros((4, 1, 3))
    U[0] = 1.0
    U[1, 0] = [1e16, 1.0, -1e16]
    U[3] = 3.0
    assert list(oracle_mod.Oracle(prm).sums(U)) == [3.0, 1.0, 0.0, 9.0]


def _feature_cases():
    prm, U0, grav = inputs.polytrope(48)
    yield "polytrope (r, z), field, floors", prm, U0, grav
    yield "shear layer", *inputs.kelvin_helmholtz(40, seed=7), None
    yield "heavy over light", *inputs.rayleigh_taylor(24, 48), None
    prm, U0 = inputs.kelvin_helmholtz(24, seed=3)
    yield "characteristic", dict(prm, recon=1), U0, None


def test_results_do_not_depend_on_thread_count(oracle_mod):
    keep = oracle_mod.threads()
    try:
        for name, prm, U0, grav in _feature_cases():
            o = oracle_mod.Oracle(prm, gravity=grav)
            out = []
            for nt in (1, 3, 8):
                oracle_mod.set_threads(nt)
                U, t, dts, als = o.run(U0, 4)
                out.append((U, t, dts, als, o.sums(U), o.alpha(U)))
            for other in out[1:]:
                for x, y in zip(out[0], other):
                    assert np.array_equal(np.asarray(x), np.asarray(y)), name
    finally:
        oracle_mod.set_threads(keep)
