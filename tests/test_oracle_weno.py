"""Pins of the oracle's WENO5 reconstruction against facts derived here, not
retyped: candidate stencils and the five-point linear scheme from polynomial
exactness, smoothness indicators from their integral definition (Jiang &
Shu 1996, the scheme cited in Sect. 2.1), all in exact rational arithmetic
with sympy."""
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

x = sp.symbols("x")


def _cell_avg_poly_coeffs(cells, target):
    """Coefficients c_j with sum_j c_j vbar_j = P(target) for every polynomial P of
    degree < len(cells), vbar_j = average of P over [j - 1/2, j + 1/2] (unit cells).
    Finite-difference WENO reconstructs the flux at a face from point values with
    exactly these weights (the point values play the role of cell averages of the
    primitive of the flux)."""
    n = len(cells)
    M = sp.zeros(n, n)
    rhs = sp.zeros(n, 1)
    for m in range(n):
        for k, j in enumerate(cells):
            M[m, k] = sp.integrate(x ** m, (x, j - sp.Rational(1, 2), j + sp.Rational(1, 2)))
        rhs[m] = sp.Rational(target) ** m if m else 1
    return list(M.solve(rhs))


def _stencils():
    half = sp.Rational(5, 2)  # face to the right of cell 2 (cells 0..4)
    cand = [_cell_avg_poly_coeffs([0, 1, 2], half), _cell_avg_poly_coeffs([1, 2, 3], half),
            _cell_avg_poly_coeffs([2, 3, 4], half)]
    big = _cell_avg_poly_coeffs([0, 1, 2, 3, 4], half)
    # linear weights d_k: sum_k d_k cand_k == big on the five cells
    d = sp.symbols("d0:3")
    eqs = []
    for j in range(5):
        tot = 0
        for k in range(3):
            if k <= j <= k + 2:
                tot += d[k] * cand[k][j - k]
        eqs.append(sp.Eq(tot, big[j]))
    sol = sp.solve(eqs, d, dict=True)[0]
    return cand, big, [sol[d[k]] for k in range(3)]


def _beta_forms():
    """beta_k(v) = sum_{l=1,2} int_{cell 2} (d^l P_k / dx^l)^2 dx (unit cells), P_k the
    quadratic whose cell averages on stencil k are the data.  Returned as sympy
    expressions in v0..v4."""
    v = sp.symbols("v0:5")
    betas = []
    for k in range(3):
        cells = [k, k + 1, k + 2]
        a = sp.symbols("a0:3")
        P = a[0] + a[1] * x + a[2] * x ** 2
        eqs = [sp.Eq(sp.integrate(P, (x, j - sp.Rational(1, 2), j + sp.Rational(1, 2))), v[j])
               for j in cells]
        sol = sp.solve(eqs, a, dict=True)[0]
        Pk = P.subs(sol)
        lo, hi = 2 - sp.Rational(1, 2), 2 + sp.Rational(1, 2)
        b = sum(sp.integrate(sp.diff(Pk, x, l) ** 2, (x, lo, hi)) for l in (1, 2))
        betas.append(sp.expand(b))
    return v, betas


@pytest.fixture(scope="module")
def derived():
    cand, big, d = _stencils()
    v, betas = _beta_forms()
    return cand, big, d, v, betas


def test_linear_weights_are_the_classical_ones(derived):
    _, _, d, _, _ = derived
    # stated as a fact to check the derivation itself
    assert d == [sp.Rational(1, 10), sp.Rational(3, 5), sp.Rational(3, 10)]


def _js_exact(vals, eps, derived):
    """Jiang-Shu weights and reconstruction in exact rational arithmetic (the inputs
    are the exact binary values of the doubles), from the derived candidates,
    linear weights and indicators."""
    cand, _, d, v, betas = derived

    def rat(f):
        fr = Fraction(f)
        return sp.Rational(fr.numerator, fr.denominator)

    sub = {v[j]: rat(vals[j]) for j in range(5)}
    q = [sum(c * sub[v[k + j]] for j, c in enumerate(cand[k])) for k in range(3)]
    b = [betas[k].subs(sub) for k in range(3)]
    e = rat(eps)
    a = [d[k] / (e + b[k]) ** 2 for k in range(3)]
    return sum(a[k] * q[k] for k in range(3)) / sum(a)


def test_nonlinear_reconstruction_matches_exact_js(oracle_mod, derived):
    rng = np.random.default_rng(11)
    for trial in range(60):
        scale = 10.0 ** rng.uniform(-3, 3)
        vals = list(scale * rng.standard_normal(5))
        if trial % 3 == 0:  # a jump inside the stencil
            vals = [vals[0], vals[0], vals[0] + 5 * scale, vals[3], vals[4]]
        eps = 1e-6 * scale ** 2 if trial % 2 else 1e-6
        exact = _js_exact(vals, eps, derived)
        got = oracle_mod.weno5(vals, eps)
        assert abs(got - float(exact)) <= 4e-15 * max(abs(float(exact)), scale), (vals, got, exact)


def test_linear_limit_is_fifth_order_exact_for_quartics(oracle_mod, derived):
    _, big, _, _, _ = derived
    rng = np.random.default_rng(3)
    for _ in range(20):
        c = rng.standard_normal(5)
        P = sum(float(c[m]) * x ** m for m in range(5))
        avgs = [float(sp.integrate(P, (x, j - 0.5, j + 0.5))) for j in range(5)]
        face = float(P.subs(x, 2.5))
        # eps -> infinity makes every weight its linear value
        got = oracle_mod.weno5(avgs, 1e30)
        lin = sum(float(big[j]) * avgs[j] for j in range(5))
        assert abs(got - face) < 1e-12 * (1 + abs(face))
        assert abs(lin - face) < 1e-12 * (1 + abs(face))


def test_quadratics_exact_for_any_weights(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(20):
        c = rng.standard_normal(3)
        P = sum(float(c[m]) * x ** m for m in range(3))
        avgs = [float(sp.integrate(P, (x, j - 0.5, j + 0.5))) for j in range(5)]
        assert abs(oracle_mod.weno5(avgs, 1e-6) - float(P.subs(x, 2.5))) < 1e-12


def test_constant_data_and_odd_symmetry(oracle_mod):
    rng = np.random.default_rng(7)
    for _ in range(50):
        v = rng.standard_normal(5) * 10 ** rng.uniform(-5, 5)
        assert oracle_mod.weno5(-v, 1e-6) == -oracle_mod.weno5(v, 1e-6)  # bitwise
        c = float(v[0])
        assert abs(oracle_mod.weno5([c] * 5, 1e-6) - c) <= 2e-16 * abs(c) * 4


def test_eno_property_across_a_jump(oracle_mod):
    # the stencil containing the jump gets (almost) no weight
    got = oracle_mod.weno5([0.0, 0.0, 0.0, 1.0, 1.0], 1e-6)
    assert abs(got) < 1e-9
    got = oracle_mod.weno5([1.0, 1.0, 0.0, 0.0, 0.0], 1e-6)
    assert abs(got) < 1e-9


def test_face_value_matches_exact_js_sum(oracle_mod, derived):
    """The face value W(f+ stencil) + W(f- stencil), formed over one common
    denominator, equals the sum of the two exact Jiang-Shu reconstructions
    within a few units in the last place of the larger term; swapping the two
    sides leaves it bit for bit unchanged, and negating both negates it."""
    rng = np.random.default_rng(13)
    for trial in range(60):
        scale = 10.0 ** rng.uniform(-3, 3)
        p = list(scale * rng.standard_normal(5))
        m = list(scale * rng.standard_normal(5))
        if trial % 3 == 0:
            p = [p[0], p[0], p[0] + 5 * scale, p[3], p[4]]
        eps = 1e-6 * scale ** 2 if trial % 2 else 1e-6
        exact = _js_exact(p, eps, derived) + _js_exact(m, eps, derived)
        got = oracle_mod.weno5_face(p, m, eps)
        ref = max(abs(float(_js_exact(p, eps, derived))), abs(float(_js_exact(m, eps, derived))), scale)
        assert abs(got - float(exact)) <= 8e-15 * ref, (p, m, got, exact)
        assert oracle_mod.weno5_face(m, p, eps) == got
        assert oracle_mod.weno5_face([-x for x in p], [-x for x in m], eps) == -got


def test_common_denominator_magnitude_domain(oracle_mod):
    """The face value over one common denominator multiplies eighth powers of
    the smoothness indicators: it is homogeneous of degree one (for stencils
    large against eps) up to split-flux magnitudes of 1e17 and overflows to
    NaN by 1e19 (by 1e18 for most stencils), the input domain include/hydro.h
    states."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        p = rng.uniform(-1, 1, 5)
        m = rng.uniform(-1, 1, 5)
        ref = oracle_mod.weno5_face(p * 1e9, m * 1e9) / 1e9
        scale = max(np.abs(p).max(), np.abs(m).max())
        for e in (6, 12, 15, 17):
            S = 10.0 ** e
            f = oracle_mod.weno5_face(p * S, m * S)
            assert np.isfinite(f) and abs(f / S - ref) <= 1e-12 * scale, (trial, e)
        assert not np.isfinite(oracle_mod.weno5_face(p * 1e19, m * 1e19)), trial
