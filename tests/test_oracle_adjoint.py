"""Pins of the reference adjoint (autograd through the plain-PyTorch step of
``oracle.torch_ref``) against central finite differences of the C oracle --
a separate writing of the forward step -- with the time step and the LF
speeds of every stage frozen at recorded values (the only non-smooth parts of
the step are those maxima, and the gradient is defined with them held
fixed)."""
import numpy as np
import pytest
import torch

from paper_1507_08549_amd import inputs

P, T, R = inputs.PERIODIC, inputs.TRANSMISSIVE, inputs.REFLECTING

CASES = {
    "kh_periodic": lambda: (inputs.kelvin_helmholtz(12, seed=7), None),
    "rt_reflecting_gravity": lambda: (inputs.rayleigh_taylor(8, 16, seed=7), None),
    "sod_1d": lambda: (inputs.sod(24), None),
    "cyl_homologous": lambda: (inputs.homologous(10, 0.4, -0.3, geometry=1), None),
    "mixed_bc": lambda: (_mixed(), None),
}


def _mixed():
    prm, U = inputs.kelvin_helmholtz(10, seed=3)
    prm["bc"] = [R, T, P, P]
    return prm, U


def _setup(name):
    (prm, U), grav = CASES[name]()
    return prm, U, grav


@pytest.mark.parametrize("name", sorted(CASES))
def test_torch_forward_matches_c_oracle(oracle_mod, name):
    from oracle import torch_ref
    prm, U, grav = _setup(name)
    o = oracle_mod.Oracle(prm, grav)
    dt = o.cfl(U)
    U1, al = o.step(U, dt)
    U1t = torch_ref.step_np(prm, grav, U, dt, al)
    assert np.abs(U1 - U1t).max() <= 1e-14 * np.abs(U1).max()


@pytest.mark.parametrize("name", sorted(CASES))
def test_reference_vjp_matches_central_differences(oracle_mod, name):
    from oracle import torch_ref
    prm, U, grav = _setup(name)
    o = oracle_mod.Oracle(prm, grav)
    dt = o.cfl(U)
    _, al = o.step(U, dt)
    rng = np.random.default_rng(1)
    lam = rng.standard_normal(U.shape)
    g = torch_ref.vjp(prm, grav, U, dt, al, lam)
    # The WENO weights vary on the scale of eps where the smoothness indicators
    # are ~eps (flat regions with small noise), so the step is smooth but
    # strongly curved there: the difference step h must be small (1e-8 of the
    # state scale) for the O(h^2) truncation error to fall below the
    # tolerance; the rounding error of the difference is then ~1e-7 relative.
    scale = np.abs(U).max(axis=(1, 2), keepdims=True)
    h = 1e-8
    for trial in range(3):
        v = rng.standard_normal(U.shape) * scale
        fp, _ = o.step(U + h * v, dt, al)
        fm, _ = o.step(U - h * v, dt, al)
        fd = np.sum(lam * (fp - fm)) / (2 * h)
        ad = np.sum(g * v)
        assert abs(fd - ad) <= 2e-6 * (abs(ad) + 1e-2 * np.abs(g * v).sum()), (fd, ad)
    # single entries
    for trial in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in U.shape)
        e = np.zeros_like(U)
        e[idx] = scale[idx[0], 0, 0]
        fp, _ = o.step(U + h * e, dt, al)
        fm, _ = o.step(U - h * e, dt, al)
        fd = np.sum(lam * (fp - fm)) / (2 * h)
        ad = g[idx] * scale[idx[0], 0, 0]
        assert abs(fd - ad) <= 2e-6 * (abs(ad) + np.abs(lam).max()), (idx, fd, ad)


def test_reference_vjp_through_several_steps(oracle_mod):
    from oracle import torch_ref
    prm, U, grav = _setup("kh_periodic")
    o = oracle_mod.Oracle(prm, grav)
    Un, _, dts, als = o.run(U, 4)
    rng = np.random.default_rng(2)
    lam = rng.standard_normal(U.shape)
    g = torch_ref.vjp_steps(prm, grav, U, dts, als, lam)

    def replay(V):
        for dt, al in zip(dts, als):
            V, _ = o.step(V, dt, al)
        return V

    v = rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2), keepdims=True)
    h = 1e-8
    fd = np.sum(lam * (replay(U + h * v) - replay(U - h * v))) / (2 * h)
    ad = np.sum(g * v)
    assert abs(fd - ad) <= 2e-6 * abs(ad), (fd, ad)


def test_reference_vjp_taylor_remainder_is_second_order(oracle_mod):
    """|J(U + h v) - J(U) - h <grad J, v>| falls as h^2 for the scalar
    J = <lam, step(U)> (on smooth data, where the asymptotic range is wide)."""
    from oracle import torch_ref
    prm, U = inputs.advection_2d(12)
    grav = None
    o = oracle_mod.Oracle(prm, grav)
    dt = o.cfl(U)
    base, al = o.step(U, dt)
    rng = np.random.default_rng(3)
    lam = rng.standard_normal(U.shape)
    g = torch_ref.vjp(prm, grav, U, dt, al, lam)
    v = rng.standard_normal(U.shape) * 1e-2
    rem = []
    for h in (6.25e-3, 3.125e-3, 1.5625e-3, 7.8125e-4):
        f, _ = o.step(U + h * v, dt, al)
        rem.append(abs(np.sum(lam * (f - base)) - h * np.sum(g * v)))
    slopes = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all((slopes > 1.85) & (slopes < 2.3)), slopes


def test_sine_mode_objective_closed_form_at_zero_steps():
    """For the shear layer with v_y = sum_k a_k sin(2 pi k x) and
    J = sum_cells m_y^2 / (2 rho) dx dy, at t = 0 the column mass is
    sum_j rho_j dy = 1.5 and the sines are orthogonal on the centres, so
    J = 0.375 sum a_k^2 and dJ/da_k = 0.75 a_k."""
    prm = inputs.kh_sine_params(128)
    a = torch.tensor(inputs.kh_sine_amplitudes(16, seed=5), dtype=torch.float64, requires_grad=True)
    U = inputs.kh_sine_state(a, prm)
    dxdy = 1.0 / (128 * 128)
    J = (0.5 * U[2] ** 2 / U[0]).sum() * dxdy
    (g,) = torch.autograd.grad(J, a)
    an = a.detach().numpy()
    assert abs(J.item() - 0.375 * np.sum(an ** 2)) < 1e-14
    assert np.allclose(g.numpy(), 0.75 * an, rtol=1e-12, atol=1e-18)


def test_float32_reference_is_single_precision(oracle_mod):
    """The float32 form of the reference adjoint (used to measure what single
    precision alone costs) runs in single precision: it differs from the
    float64 form by far more than float64 rounding and by far less than the
    result itself, and the float64 form is unchanged by the option."""
    import torch

    from oracle import torch_ref
    prm, U0 = inputs.kelvin_helmholtz(24, seed=9)
    o = oracle_mod.Oracle(prm)
    dt = o.cfl(U0)
    _, al = o.step(U0, dt)
    lam = np.random.default_rng(8).standard_normal(U0.shape)
    w64 = torch_ref.vjp(prm, None, U0, dt, al, lam)
    assert np.array_equal(w64, torch_ref.vjp(prm, None, U0, dt, al, lam, dtype=torch.float64))
    w32 = torch_ref.vjp(prm, None, U0, dt, al, lam, dtype=torch.float32)
    err = np.abs(w32 - w64).sum() / np.abs(w64).sum()
    assert 1e-9 < err < 1e-2, err
