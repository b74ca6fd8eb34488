"""The allocation-free step (hydro_step_noalloc, for callers that cannot
allocate device memory) against the context step (hydro_step) it varies:
the same kernels, so the same state bit for bit.  Two calls in a row on one
device, the second on a smaller grid (the scratch array keeps the first call's
contents), in FP64 and FP32-bulk, with computed and with replayed LF speeds,
with a gravity field, cylindrical geometry and floors; the unphysical flag;
a capacity-sized grid."""
import numpy as np
import pytest

from paper_1507_08549_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def hydro():
    from paper_1507_08549_amd import hydro as h
    return h


def _both(torch, hydro, prm, U0, grav, precision, alpha, steps=2):
    """The state after `steps` steps by hydro_step and by hydro_step_noalloc."""
    g = None if grav is None else torch.tensor(grav, dtype=torch.float64, device="cuda")
    s = hydro.Solver(prm, gravity=g, precision=precision)
    Ua = torch.tensor(U0, dtype=torch.float64, device="cuda")
    Ub = Ua.clone()
    flag = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    dt = s.cfl(Ua)
    for _ in range(steps):
        s.step(Ua, dt, alpha=alpha)
        hydro.step_noalloc(prm, Ub, dt, alpha=alpha, gravity=g, precision=precision, unphysical=flag)
    s.check()
    s.close()
    torch.cuda.synchronize()
    return Ua.cpu().numpy(), Ub.cpu().numpy(), int(flag.item())


@pytest.mark.parametrize("precision", [0, 1])
def test_two_calls_second_smaller(torch, hydro, precision):
    big_prm, big_U = inputs.kelvin_helmholtz(96, seed=3)
    a, b, f = _both(torch, hydro, big_prm, big_U, None, precision, None)
    print(f"96^2 shear layer, precision {precision}: max |diff| {np.abs(a - b).max():.3e}", flush=True)
    assert f == 0 and np.array_equal(a, b)
    prm, U0 = inputs.rayleigh_taylor(24, 40)
    a, b, f = _both(torch, hydro, prm, U0, None, precision, None)
    print(f"24 x 40 heavy-over-light layer, precision {precision}: max |diff| {np.abs(a - b).max():.3e}",
          flush=True)
    assert f == 0 and np.array_equal(a, b)


def test_field_gravity_cylindrical_floors_replayed_speeds(torch, hydro):
    prm, U0, grav = inputs.polytrope(64)
    alpha = np.array([[1.3, 1.2], [1.31, 1.21], [1.29, 1.19]])
    for n_prm, n_U, n_g in ((prm, U0, grav), inputs.polytrope(40)):
        a, b, f = _both(torch, hydro, n_prm, n_U, n_g, 0, alpha)
        assert f == 0 and np.array_equal(a, b)
        a, b, f = _both(torch, hydro, n_prm, n_U, n_g, 0, None)
        assert f == 0 and np.array_equal(a, b)


def test_characteristic_reconstruction(torch, hydro):
    prm, U0 = inputs.kelvin_helmholtz(48, seed=5)
    prm = dict(prm, recon=hydro.CHARACTERISTIC)
    a, b, f = _both(torch, hydro, prm, U0, None, 0, None)
    assert f == 0 and np.array_equal(a, b)


def test_unphysical_flag_is_reported(torch, hydro):
    prm, U0 = inputs.kelvin_helmholtz(32, seed=1)
    U0 = U0.copy()
    U0[3, 5, 7] = 0.01  # internal energy negative: p < 0 in one cell
    U = torch.tensor(U0, dtype=torch.float64, device="cuda")
    flag = torch.zeros((1,), dtype=torch.int32, device="cuda")
    hydro.step_noalloc(prm, U, 1e-4, alpha=[[3.0, 3.0]] * 3, unphysical=flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 1
    # the next call starts from a cleared flag
    prm2, U2 = inputs.kelvin_helmholtz(32, seed=2)
    V = torch.tensor(U2, dtype=torch.float64, device="cuda")
    hydro.step_noalloc(prm2, V, 1e-4, unphysical=flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0


def test_capacity_sized_grid(torch, hydro):
    prm, U0 = inputs.kelvin_helmholtz(1024, seed=2)
    assert prm["nx"] * prm["ny"] == hydro.NOALLOC_MAX_CELLS
    a, b, f = _both(torch, hydro, prm, U0, None, 0, None, steps=1)
    assert f == 0 and np.array_equal(a, b)
    with pytest.raises(hydro.HydroError):
        big_prm = dict(prm, nx=1025)
        hydro.step_noalloc(big_prm, torch.zeros((4, 1024, 1025), dtype=torch.float64, device="cuda"), 1e-4)
