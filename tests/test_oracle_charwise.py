"""Pins of the oracle's characteristic-wise reconstruction (the "WENO-Roe"
variant of Sect. 2.1: the split fluxes are reconstructed in the eigenvector
fields of the flux Jacobian at the Roe average of the two cells beside each
face).

* the eigenvectors: L R = I, R diag(u_n - c, u_n, u_n, u_n + c) L equals the
  flux Jacobian (central differences of the flux), and at two different
  states the Roe property A_roe (U_r - U_l) = F(U_r) - F(U_l) holds (this pins
  the averaged velocity, enthalpy and sound speed);
* fifth-order convergence on smooth advection in 1D and 2D;
* conservation to round-off, uniform flow and the x/y transpose bit for bit;
* on the shock tubes of Table Test1D and Sod, the spurious oscillations
  (total variation above the exact solution's) are at most a quarter of the
  component-wise scheme's: the purpose of the characteristic projection.
"""
import numpy as np
import pytest

from exact_riemann import RiemannSolution
from paper_1507_08549_amd import inputs

P, T, R = inputs.PERIODIC, inputs.TRANSMISSIVE, inputs.REFLECTING
G = 1.4


def _cons(rho, u, v, p, g=G):
    return np.array([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])


def _flux(U, d, g=G):
    r, mx, my, E = U
    u, v = mx / r, my / r
    p = (g - 1) * (E - 0.5 * (mx * u + my * v))
    if d == 0:
        return np.array([mx, mx * u + p, my * u, (E + p) * u])
    return np.array([my, mx * v, my * v + p, (E + p) * v])


def _perm(d):
    # rotated frame (rho, m_n, m_t, E) -> original components
    return [0, 1, 2, 3] if d == 0 else [0, 2, 1, 3]


@pytest.mark.parametrize("d", [0, 1])
def test_eigenvectors_and_roe_property(oracle_mod, d):
    rng = np.random.default_rng(3 + d)
    for _ in range(20):
        rho, u, v, p = rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.1, 5)
        U = _cons(rho, u, v, p)
        L, Rm = oracle_mod.char_eig(U, U, d, G)
        np.testing.assert_allclose(L @ Rm, np.eye(4), atol=1e-13)
        c = np.sqrt(G * p / rho)
        un = u if d == 0 else v
        lam = np.diag([un - c, un, un, un + c])
        h = 1e-6 * np.maximum(np.abs(U), 1.0)
        J = np.stack([(_flux(U + h[k] * e, d) - _flux(U - h[k] * e, d)) / (2 * h[k])
                      for k, e in enumerate(np.eye(4))], axis=1)
        pm = _perm(d)
        Jrot = J[np.ix_(pm, pm)]
        np.testing.assert_allclose(Rm @ lam @ L, Jrot, rtol=0, atol=1e-7 * np.abs(Jrot).max())
        # Roe property between two different states
        U2 = _cons(rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.1, 5))
        L2, R2 = oracle_mod.char_eig(U, U2, d, G)
        wl = U[0] ** 0.5
        wr = U2[0] ** 0.5
        unl = (U[1 + d] / U[0])
        unr = (U2[1 + d] / U2[0])
        un_roe = (wl * unl + wr * unr) / (wl + wr)
        c_roe = (R2[1, 3] - R2[1, 0]) / 2
        A = R2 @ np.diag([un_roe - c_roe, un_roe, un_roe, un_roe + c_roe]) @ L2
        dF = (_flux(U2, d) - _flux(U, d))[pm]
        np.testing.assert_allclose(A @ (U2 - U)[pm], dF, rtol=0, atol=1e-12 * np.abs(dF).max())


def _advect_1d(oracle_mod, n, t_end=1.0):
    prm, U = inputs.advection_1d(n)
    prm["recon"] = 1
    o = oracle_mod.Oracle(prm)
    dt = 0.5 * (1.0 / n) ** (5.0 / 3.0)
    nst = int(np.ceil(t_end / dt))
    dt = t_end / nst
    for _ in range(nst):
        U, _ = o.step(U, dt)
    x, _ = inputs.centres(prm)
    return np.abs(U[0, 0] - (1 + 0.2 * np.sin(2 * np.pi * (x - t_end)))).mean()


def test_fifth_order_smooth_advection_1d(oracle_mod):
    errs = [_advect_1d(oracle_mod, n) for n in (32, 64, 128)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.8), orders


def test_fifth_order_smooth_advection_2d(oracle_mod):
    errs = []
    t_end = 0.25
    for n in (16, 32, 64):
        prm, U = inputs.advection_2d(n)
        prm["recon"] = 1
        o = oracle_mod.Oracle(prm)
        dt = 0.25 * (1.0 / n) ** (5.0 / 3.0)
        nst = int(np.ceil(t_end / dt))
        dt = t_end / nst
        for _ in range(nst):
            U, _ = o.step(U, dt)
        x, y = inputs.centres(prm)
        X, Y = np.meshgrid(x, y)
        errs.append(np.abs(U[0] - (1 + 0.2 * np.sin(2 * np.pi * (X + Y - 2 * t_end)))).mean())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > 4.6, (errs, orders)


def _random_state(ny, nx, seed):
    rng = np.random.default_rng(seed)
    return inputs.state_from_primitive(1.0 + 0.5 * rng.uniform(0, 1, (ny, nx)),
                                       0.5 * rng.uniform(-1, 1, (ny, nx)),
                                       0.5 * rng.uniform(-1, 1, (ny, nx)),
                                       1.0 + 0.5 * rng.uniform(0, 1, (ny, nx)), G)


def test_conservation_and_uniform_flow(oracle_mod):
    prm = inputs.make_params(24, 20, 0.0, 1.0, 0.0, 1.0, [P] * 4, G)
    prm["recon"] = 1
    o = oracle_mod.Oracle(prm)
    U = _random_state(20, 24, 1)
    s0 = U.reshape(4, -1).sum(axis=1)
    for _ in range(5):
        U, _ = o.step(U, 0.002)
    s1 = U.reshape(4, -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) <= 1e-13 * np.abs(U).reshape(4, -1).sum(axis=1))
    Uu = np.broadcast_to(_cons(1.3, 0.4, -0.2, 0.9)[:, None, None], (4, 20, 24)).copy()
    V, _ = o.step(Uu, 0.01)
    assert np.array_equal(V, Uu)


@pytest.mark.parametrize("bc", [(P, P, P, P), (R, T, T, R)])
def test_transpose_symmetry_bitwise(oracle_mod, bc):
    n = 16
    prm = inputs.make_params(n, n, 0.0, 1.0, 0.0, 1.0, list(bc), G)
    prmT = inputs.make_params(n, n, 0.0, 1.0, 0.0, 1.0, [bc[2], bc[3], bc[0], bc[1]], G)
    prm["recon"] = prmT["recon"] = 1
    U = _random_state(n, n, 2)
    UT = np.stack([U[0].T, U[2].T, U[1].T, U[3].T])
    a, _ = oracle_mod.Oracle(prm).step(U, 0.003)
    b, _ = oracle_mod.Oracle(prmT).step(UT, 0.003)
    assert np.array_equal(np.stack([b[0].T, b[2].T, b[1].T, b[3].T]), a)


def _tv_excess(oracle_mod, st, x0, t, recon, n=400):
    prm, U = inputs.riemann_1d(*st, x0=x0, n=n, cfl=0.5)
    prm["recon"] = recon
    U2, tt, _, _ = oracle_mod.Oracle(prm).run(U, 100000, t_end=t)
    assert tt == t
    x, _ = inputs.centres(prm)
    ex = RiemannSolution(*st).sample((x - x0) / t)
    rho = U2[0, 0]
    return np.abs(np.diff(rho)).sum() - np.abs(np.diff(ex[0])).sum(), np.abs(rho - ex[0]).mean()


def _rows():
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    return np.loadtxt(os.path.join(here, "golden", "riemann_table_test1d.txt"))


@pytest.mark.parametrize("case", ["sod", 0, 2, 3])
def test_fewer_oscillations_at_shocks(oracle_mod, case):
    if case == "sod":
        st, x0, t = (1.0, 0.0, 1.0, 0.125, 0.0, 0.1), 0.5, 0.2
    else:
        r = _rows()[case]
        st, x0, t = tuple(r[3:]), r[2], r[1]
    comp, e0 = _tv_excess(oracle_mod, st, x0, t, 0)
    char, e1 = _tv_excess(oracle_mod, st, x0, t, 1)
    assert comp > 0 and char < 0.25 * comp, (comp, char)
    assert e1 < 1.1 * e0, (e0, e1)  # no loss of accuracy
