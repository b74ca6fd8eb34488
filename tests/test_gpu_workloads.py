"""The two-dimensional and one-dimensional test problems of Sect. 5.1-5.2 on
the GPU path: the shock tubes of Table Test1D at the paper's 2000 cells, the
Blast test's x and y mirror symmetry and the Explosion test's x = y symmetry
(both claimed in Sect. 5.2; exact here because the arithmetic is written to be
equivariant), and the Gresho vortex error table (Table Test2D_test1) as
context."""
import os

import numpy as np
import pytest

from paper_1507_08549_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.fixture(scope="module")
def hydro():
    from paper_1507_08549_amd import hydro as _h
    _h.load()
    return _h


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("row", range(4))
def test_table_test1d_tubes_at_2000_cells(torch, hydro, oracle_mod, row):
    from exact_riemann import RiemannSolution
    r = np.loadtxt(os.path.join(HERE, "golden", "riemann_table_test1d.txt"))[row]
    t0, x0, st = r[1], r[2], tuple(r[3:])
    prm, U0 = inputs.riemann_1d(*st, x0=x0, n=2000, cfl=0.5)
    want, t, dts, _ = oracle_mod.Oracle(prm).run(U0, 10 ** 6, t_end=t0)
    s = hydro.Solver(prm)
    U = _dev(torch, U0)
    k, t_gpu, _, _ = s.run(U, len(dts) + 10, t_end=t0)
    got = U.cpu().numpy()
    assert k == len(dts) and t_gpu == t
    assert np.array_equal(got, want)
    x, _ = inputs.centres(prm)
    ex = RiemannSolution(*st).sample((x - x0) / t0)
    rho = got[0, 0]
    assert np.abs(rho - ex[0]).mean() < 0.1 * np.abs(ex[0]).mean()


def _mirror_x(U):
    M = U[:, :, ::-1].copy()
    M[1] *= -1
    return M


def _mirror_y(U):
    M = U[:, ::-1, :].copy()
    M[2] *= -1
    return M


def test_blast_keeps_both_mirror_symmetries(torch, hydro):
    prm, U0 = inputs.blast(512, 768)
    assert np.array_equal(U0, _mirror_x(U0)) and np.array_equal(U0, _mirror_y(U0))
    s = hydro.Solver(prm)
    U = _dev(torch, U0)
    s.run(U, 300)
    got = U.cpu().numpy()
    assert np.array_equal(got, _mirror_x(got))
    assert np.array_equal(got, _mirror_y(got))
    assert not np.array_equal(got, U0)


def test_explosion_keeps_diagonal_symmetry(torch, hydro):
    prm, U0 = inputs.explosion(512)
    T = lambda U: np.ascontiguousarray(U[[0, 2, 1, 3]].transpose(0, 2, 1))
    assert np.array_equal(U0, T(U0))
    s = hydro.Solver(prm)
    U = _dev(torch, U0)
    s.run(U, 300)
    got = U.cpu().numpy()
    assert np.array_equal(got, T(got))


def test_blast_first_steps_match_oracle(torch, hydro, oracle_mod):
    prm, U0 = inputs.blast(512, 768)
    want, _, _, _ = oracle_mod.Oracle(prm).run(U0, 2)
    U = _dev(torch, U0)
    hydro.Solver(prm).run(U, 2)
    assert np.array_equal(U.cpu().numpy(), want)


def test_gresho_50_matches_oracle_to_t3(torch, hydro, oracle_mod):
    prm, U0 = inputs.gresho(50)
    want, t, dts, _ = oracle_mod.Oracle(prm).run(U0, 10 ** 6, t_end=3.0)
    U = _dev(torch, U0)
    k, t_gpu, _, _ = hydro.Solver(prm).run(U, len(dts) + 10, t_end=3.0)
    assert k == len(dts) and t_gpu == 3.0
    assert np.array_equal(U.cpu().numpy(), want)


def test_gresho_error_table(torch, hydro):
    """Errors at t = 3 for the four resolutions of Table Test2D_test1.  The
    paper's scheme differs (5-stage RK3), so its numbers are context: the
    test checks the L1 pressure error falls with resolution and is of the
    paper's magnitude on the coarsest grid (within a factor 4)."""
    paper = np.loadtxt(os.path.join(HERE, "golden", "gresho_table_test2d.txt"))
    rows = []
    for n in (50, 100, 200, 400):
        prm, U0 = inputs.gresho(n)
        s = hydro.Solver(prm)
        U = _dev(torch, U0)
        s.run(U, 10 ** 6, t_end=3.0)
        got = U.cpu().numpy()
        s0, s1 = s.sums(_dev(torch, U0)), s.sums(U)
        p0 = inputs.primitive_from_state(U0, 1.4)[3]
        p1 = inputs.primitive_from_state(got, 1.4)[3]
        rows.append((abs(s1[0] - s0[0]) / s0[0], abs(s1[3] - s0[3]) / s0[3],
                     np.abs(p1 - p0).sum() / (n * n)))
    rows = np.array(rows)
    print("\nGresho t = 3: n, dM/M, dE/E, L1(p) (SSP-RK3 here | paper)")
    for n, r, pr in zip((50, 100, 200, 400), rows, paper):
        print(f"{n:4d} {r[0]:.2e} {r[1]:.2e} {r[2]:.2e} | {pr[3]:.2e} {pr[4]:.2e} {pr[5]:.2e}")
    assert np.all(np.diff(rows[:, 2]) < 0), rows
    assert 0.25 < rows[0, 2] / paper[0, 5] < 4.0
