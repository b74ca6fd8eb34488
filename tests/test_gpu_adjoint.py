"""GPU parity of the hand-written adjoint (hydro_step_vjp) against the
reference adjoint: autograd through the plain-PyTorch FP64 step of the oracle
package (itself pinned against central differences of the C oracle).

The adjoint is not bit-exact (its sums run in a different order than
autograd's).  Every test prints its error; the bounds are about three times
the largest error measured (the adjoint's arithmetic has a fixed order, so the
errors are the same on every run):

* FP64 stage adjoint, relative L1 error of the whole vector: on random states
  largest measured 2.8e-14 (the 1024^2 sine-mode shear layer; 2.2e-14 for the
  300-cell tube, <= 1.4e-14 on every small grid, boundary set and geometry),
  bound 8e-14.  On shear-layer states with flat layers and cell noise, 1.1e-12
  to 1.2e-12 on every grid and boundary set, bound 3.5e-12: there the
  smoothness indicators are ~0, the weight derivatives carry factors up to
  1/(eps + beta) ~ 1e6, and the rounding differences of two FP64 summation
  orders grow by that much.
  FP64 rollout gradient (64^2, 24 steps): 4.6e-16 of its largest component,
  bound 1e-15.
* FP32-bulk: what single precision alone costs is measured in each test by
  evaluating the same reference in float32 (inputs rounded, every operation
  and its autograd in single precision).  The device's FP32-bulk adjoint,
  which keeps the state and the stage combination in FP64, must be no less
  accurate than that: stage adjoint 3.7e-4 against 4.6e-4 on the 48^2 shear
  layer (flat layers: the weight derivatives act on smoothness indicators of
  nearly equal neighbours, which single precision resolves to a few digits),
  1.1e-5 against 1.3e-5 on the 64 x 128 walled box; rollout gradient 1.2e-7
  against 4.2e-7, and within 3.7e-7 (three times the measured).
"""
import numpy as np
import pytest

from paper_1507_08549_amd import inputs

pytestmark = pytest.mark.gpu

P, T, R = inputs.PERIODIC, inputs.TRANSMISSIVE, inputs.REFLECTING
FP64_BOUND = 8e-14
FP64_FLAT_BOUND = 3.5e-12
FP64_ROLLOUT_BOUND = 1e-15
FP32_ROLLOUT_BOUND = 3.7e-7


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


def _random_state(ny, nx, seed, gamma=1.4):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.5 * rng.uniform(0, 1, (ny, nx))
    u = 0.5 * rng.uniform(-1, 1, (ny, nx))
    v = 0.5 * rng.uniform(-1, 1, (ny, nx))
    p = 1.0 + 0.5 * rng.uniform(0, 1, (ny, nx))
    return inputs.state_from_primitive(rho, u, v, p, gamma)


def _rel_l1(got, want):
    return np.abs(got - want).sum() / max(np.abs(want).sum(), 1e-300)


BCS = [[P, P, P, P], [T, T, T, T], [R, R, R, R], [R, T, R, T], [T, R, P, P]]
# (a cylindrical grid's axis is reflecting, never periodic)
BC_GEOMETRY = [(bc, geo) for geo in (0, 1) for bc in BCS if not (geo == 1 and bc[0] == P)]
# (116, 58): lines of exactly two and one 58-cell tiles (the ghost points of
# the last tile's line are its last three lanes)
# (3, 5): lines shorter than a stencil (periodic lines wrap more than once)
# (64, 128): both passes launch a multiple of 8 workgroups (48 and 32), so the
# tiles are handed to the XCDs in contiguous runs rather than in launch order
SHAPES = [(3, 5), (8, 8), (11, 13), (17, 33), (40, 70), (70, 130), (116, 58), (64, 128)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("bc, geometry", BC_GEOMETRY,
                         ids=lambda x: "".join("PTR"[k] for k in x) if isinstance(x, list) else ["cart", "cyl"][x])
def test_step_vjp_matches_reference(torch, hydro, oracle_mod, shape, bc, geometry):
    from oracle import torch_ref
    ny, nx = shape
    xlo = 0.0 if geometry == 1 else -0.3
    prm = inputs.make_params(nx, ny, xlo, xlo + 1.0, 0.0, 0.8, bc, 1.4, geometry=geometry,
                             gx=0.05, gy=-0.1)
    U0 = _random_state(ny, nx, seed=nx + 7 * ny)
    o = oracle_mod.Oracle(prm)
    dt = o.cfl(U0)
    _, al = o.step(U0, dt)
    lam = np.random.default_rng(3).standard_normal(U0.shape)
    want = torch_ref.vjp(prm, None, U0, dt, al, lam)
    s = hydro.Solver(prm)
    got = s.step_vjp(_dev(torch, U0), dt, al, _dev(torch, lam)).cpu().numpy()
    err = _rel_l1(got, want)
    print(f"ADJ fp64 step {ny}x{nx} bc {bc} geometry {geometry}: {err:.3e}", flush=True)
    assert err <= FP64_BOUND, err


def test_step_vjp_full_size(torch, hydro, oracle_mod):
    """The adjoint workload's grid (sine-mode shear layer, 1024^2: 18 tiles of
    58 cells along every line, lines in many workgroups), one step, against
    the reference adjoint (about ten seconds and 10 GB of host memory)."""
    from oracle import torch_ref
    prm = inputs.kh_sine_params(1024)
    U0 = inputs.kh_sine_state(inputs.kh_sine_amplitudes(), prm)
    o = oracle_mod.Oracle(prm)
    dt = o.cfl(U0)
    _, al = o.step(U0, dt)
    lam = np.random.default_rng(3).standard_normal(U0.shape)
    want = torch_ref.vjp(prm, None, U0, dt, al, lam)
    got = hydro.Solver(prm).step_vjp(_dev(torch, U0), dt, al, _dev(torch, lam)).cpu().numpy()
    err = _rel_l1(got, want)
    print(f"ADJ fp64 step 1024x1024 sine-mode shear layer: {err:.3e}", flush=True)
    assert err <= FP64_BOUND


@pytest.mark.parametrize("bc", BCS, ids=lambda b: "".join("PTR"[k] for k in b))
@pytest.mark.parametrize("n, seed", [(40, 13), (64, 2), (48, 9)])
def test_step_vjp_flat_layers(torch, hydro, oracle_mod, bc, n, seed):
    """Shear-layer states, whose layers are flat: there the smoothness
    indicators are ~0, the weight derivatives carry factors up to
    1/(eps + beta) ~ 1e6, and rounding differences between two FP64 orders of
    summation grow by that much."""
    from oracle import torch_ref
    prm, U0 = inputs.kelvin_helmholtz(n, seed=seed)
    prm["bc"] = list(bc)
    o = oracle_mod.Oracle(prm)
    dt = o.cfl(U0)
    _, al = o.step(U0, dt)
    lam = np.random.default_rng(4).standard_normal(U0.shape)
    want = torch_ref.vjp(prm, None, U0, dt, al, lam)
    got = hydro.Solver(prm).step_vjp(_dev(torch, U0), dt, al, _dev(torch, lam)).cpu().numpy()
    err = _rel_l1(got, want)
    print(f"ADJ fp64 flat-layer step {n}^2 seed {seed} bc {bc}: {err:.3e}", flush=True)
    assert err <= FP64_FLAT_BOUND


@pytest.mark.parametrize("n", [7, 300], ids=lambda n: f"n{n}")
def test_step_vjp_1d(torch, hydro, oracle_mod, n):
    from oracle import torch_ref
    prm, U0 = inputs.riemann_1d(1.0, 0.75, 1.0, 0.125, 0.0, 0.1, x0=0.3, n=n, cfl=0.5)
    prm["bc"] = [R, T, T, T]
    o = oracle_mod.Oracle(prm)
    U0, _, _, _ = o.run(U0, 3)
    dt = o.cfl(U0)
    _, al = o.step(U0, dt)
    lam = np.random.default_rng(5).standard_normal(U0.shape)
    want = torch_ref.vjp(prm, None, U0, dt, al, lam)
    got = hydro.Solver(prm).step_vjp(_dev(torch, U0), dt, al, _dev(torch, lam)).cpu().numpy()
    err = _rel_l1(got, want)
    print(f"ADJ fp64 step 1D n={n}: {err:.3e}", flush=True)
    assert err <= FP64_BOUND


def test_step_vjp_gravity_field(torch, hydro, oracle_mod):
    """A gravity field (that of the n = 3 polytrope) acting on a dense random
    state in cylindrical geometry (the adjoint is defined without floors)."""
    from oracle import torch_ref
    prm, _, g = inputs.polytrope(40, seed=4)
    prm["rho_floor"] = 0.0
    prm["p_floor"] = 0.0
    U0 = _random_state(40, 40, seed=12, gamma=prm["gamma"])
    o = oracle_mod.Oracle(prm, g)
    dt = o.cfl(U0)
    _, al = o.step(U0, dt)
    lam = np.random.default_rng(6).standard_normal(U0.shape)
    want = torch_ref.vjp(prm, g, U0, dt, al, lam)
    s = hydro.Solver(prm, gravity=_dev(torch, g))
    got = s.step_vjp(_dev(torch, U0), dt, al, _dev(torch, lam)).cpu().numpy()
    err = _rel_l1(got, want)
    print(f"ADJ fp64 step gravity field: {err:.3e}", flush=True)
    assert err <= FP64_BOUND


@pytest.mark.parametrize("case", ["kh48", "walls64x128"])
def test_step_vjp_fp32_bulk(torch, hydro, oracle_mod, case):
    """FP32-bulk stage adjoint against the FP64 reference.  walls64x128: both
    passes launch a multiple of 8 workgroups (48 and 16: 16 columns per y
    workgroup in this form) on a grid with reflecting and transmissive edges."""
    from oracle import torch_ref
    if case == "kh48":
        prm, U0 = inputs.kelvin_helmholtz(48, seed=9)
    else:
        prm = inputs.make_params(128, 64, 0.0, 1.0, 0.0, 0.5, [R, T, R, T], 1.4, gy=-0.1)
        U0 = _random_state(64, 128, seed=21)
    o = oracle_mod.Oracle(prm)
    U0, _, _, _ = o.run(U0, 5)
    dt = o.cfl(U0)
    _, al = o.step(U0, dt)
    lam = np.random.default_rng(8).standard_normal(U0.shape)
    want = torch_ref.vjp(prm, None, U0, dt, al, lam)
    # what single precision alone costs: the same reference evaluated in float32
    e_prec = _rel_l1(torch_ref.vjp(prm, None, U0, dt, al, lam, dtype=torch.float32), want)
    s = hydro.Solver(prm, precision=hydro.FP32_BULK)
    got = s.step_vjp(_dev(torch, U0), dt, al, _dev(torch, lam)).cpu().numpy()
    err = _rel_l1(got, want)
    print(f"ADJ fp32 step {case}: device {err:.3e}, float32 reference {e_prec:.3e}", flush=True)
    assert err <= e_prec, (err, e_prec)


def test_floors_rejected_by_vjp(torch, hydro):
    prm, U0, g = inputs.polytrope(16, seed=4)
    s = hydro.Solver(prm, gravity=_dev(torch, g))
    U = _dev(torch, U0)
    with pytest.raises(hydro.HydroError):
        s.step_vjp(U, 1e-3, np.ones((3, 2)), torch.zeros_like(U))


def _objective(torch, U, prm):
    dxdy = (prm["xhi"] - prm["xlo"]) / prm["nx"] * (prm["yhi"] - prm["ylo"]) / prm["ny"]
    return (0.5 * U[2] * U[2] / U[0]).sum() * dxdy


def test_rollout_gradient_matches_reference_and_differences(torch, hydro, oracle_mod):
    """Sine-mode shear layer on 64^2, 24 steps, checkpoints every 5: the gradient
    of the final y-kinetic energy with respect to the 8 mode amplitudes, against
    (a) the reference adjoint through the oracle's own recorded schedule and
    (b) central differences of the device forward replaying the recorded
    schedule."""
    from oracle import torch_ref
    from paper_1507_08549_amd.autograd import rollout
    n, K, steps = 64, 8, 24
    prm = inputs.kh_sine_params(n)
    a_np = inputs.kh_sine_amplitudes(K, seed=5) * 20.0
    a = torch.tensor(a_np, dtype=torch.float64, device="cuda", requires_grad=True)
    s = hydro.Solver(prm)
    U0 = inputs.kh_sine_state(a, prm)
    UN = rollout(U0, s, steps, ckpt_every=5)
    J = _objective(torch, UN, prm)
    (g,) = torch.autograd.grad(J, a)
    g = g.cpu().numpy()

    # (a) reference: oracle schedule, autograd through the torch step, chain to a
    o = oracle_mod.Oracle(prm)
    U0n = inputs.kh_sine_state(a_np, prm)
    UNo, _, dts, als = o.run(U0n, steps)
    ta = torch.tensor(a_np, dtype=torch.float64, requires_grad=True)
    x = inputs.kh_sine_state(ta, prm)
    y = x
    for dt, al in zip(dts, als):
        y = torch_ref.step(prm, None, y, float(dt), [tuple(map(float, r)) for r in al])
    Jr = _objective(torch, y, prm)
    (gr,) = torch.autograd.grad(Jr, ta)
    gr = gr.numpy()
    assert abs(J.item() - Jr.item()) <= 1e-13 * abs(Jr.item())
    print(f"ADJ fp64 rollout 64^2 24 steps: max |g - g_ref| / max |g_ref| {np.abs(g - gr).max() / np.abs(gr).max():.3e}",
          flush=True)
    assert np.abs(g - gr).max() <= FP64_ROLLOUT_BOUND * np.abs(gr).max(), (g, gr)

    # (b) central differences of the device forward with the frozen schedule
    def J_of(avec):
        U = inputs.kh_sine_state(torch.tensor(avec, dtype=torch.float64, device="cuda"), prm).contiguous()
        for dt, al in zip(dts, als):
            s.step(U, float(dt), alpha=al)
        return _objective(torch, U, prm).item()

    h = 1e-7
    for k in (0, 3, 7):
        e = np.zeros(K)
        e[k] = h
        fd = (J_of(a_np + e) - J_of(a_np - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * np.abs(g).max(), (k, fd, g[k])


def test_fp32_bulk_rollout_gradient(torch, hydro, oracle_mod):
    """The sine-mode shear layer on 64^2, 24 steps, checkpoints every 5, in
    FP32-bulk: the gradient of the final y-kinetic energy with respect to the 8
    mode amplitudes against the FP64 reference gradient (autograd through the
    plain-PyTorch step along the oracle's schedule), beside what single
    precision alone costs (the same reference evaluated in float32)."""
    from oracle import torch_ref
    from paper_1507_08549_amd.autograd import rollout
    n, K, steps = 64, 8, 24
    prm = inputs.kh_sine_params(n)
    a_np = inputs.kh_sine_amplitudes(K, seed=5) * 20.0
    o = oracle_mod.Oracle(prm)
    _, _, dts, als = o.run(inputs.kh_sine_state(a_np, prm), steps)

    def ref_grad(dtype):
        ta = torch.tensor(a_np, dtype=torch.float64, requires_grad=True)
        y = inputs.kh_sine_state(ta, prm).to(dtype)
        for dt, al in zip(dts, als):
            y = torch_ref.step(prm, None, y, float(dt), [tuple(map(float, r)) for r in al])
        (g,) = torch.autograd.grad(_objective(torch, y, prm), ta)
        return g.double().numpy()

    g64, g32 = ref_grad(torch.float64), ref_grad(torch.float32)
    s = hydro.Solver(prm, precision=hydro.FP32_BULK)
    a = torch.tensor(a_np, dtype=torch.float64, device="cuda", requires_grad=True)
    UN = rollout(inputs.kh_sine_state(a, prm), s, steps, ckpt_every=5)
    (g,) = torch.autograd.grad(_objective(torch, UN, prm), a)
    g = g.cpu().numpy()
    err = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    e_prec = np.linalg.norm(g32 - g64) / np.linalg.norm(g64)
    print(f"ADJ fp32 rollout 64^2 24 steps: device {err:.3e}, float32 reference {e_prec:.3e}", flush=True)
    assert err <= e_prec and err <= FP32_ROLLOUT_BOUND, (err, e_prec)


def test_saved_stage_states_reproduce_step_and_vjp(torch, hydro, oracle_mod):
    """hydro_step_save gives the same step as hydro_step and its stage states make
    hydro_step_vjp_saved reproduce hydro_step_vjp bit for bit (same kernels,
    same inputs); U1 is the first Runge-Kutta stage of the oracle step."""
    from oracle import torch_ref
    prm, U0 = inputs.kelvin_helmholtz(40, seed=13)
    prm["bc"] = [R, T, P, P]
    o = oracle_mod.Oracle(prm)
    dt = o.cfl(U0)
    want, al = o.step(U0, dt)
    s = hydro.Solver(prm)
    U = _dev(torch, U0)
    U1 = torch.empty_like(U)
    U2 = torch.empty_like(U)
    out = torch.empty_like(U)
    s.step_save(U, dt, al, U1, U2, out=out)  # out of place
    assert np.array_equal(out.cpu().numpy(), want) and np.array_equal(U.cpu().numpy(), U0)
    s.step_save(U, dt, al, U1, U2)  # in place
    assert np.array_equal(U.cpu().numpy(), want)
    # first stage: U + dt L(U) with the oracle's own operator
    L = o.rhs(U0, al[0, 0], al[0, 1])
    assert np.abs(U1.cpu().numpy() - (U0 + dt * L)).max() <= 1e-14 * np.abs(U0).max()
    lam = _dev(torch, np.random.default_rng(4).standard_normal(U0.shape))
    a = s.step_vjp(_dev(torch, U0), dt, al, lam)
    b = s.step_vjp_saved(_dev(torch, U0), U1, U2, dt, al, lam)
    assert torch.equal(a, b)
    ref = torch_ref.vjp(prm, None, U0, dt, al, lam.cpu().numpy())
    err = _rel_l1(b.cpu().numpy(), ref)
    print(f"ADJ fp64 saved-state step, 40^2 shear layer: {err:.3e}", flush=True)
    assert err <= FP64_FLAT_BOUND


def test_run_save_keeps_every_state(torch, hydro, oracle_mod):
    """hydro_run_save: the same final state and schedule as hydro_run, each
    step's start state equal to the oracle's, its stage states equal to what
    hydro_step_save writes; stopping at t_end leaves the last state in U."""
    prm, U0 = inputs.kelvin_helmholtz(48, seed=17)
    prm["bc"] = [R, T, P, P]
    s = hydro.Solver(prm)
    n = 7
    U = _dev(torch, U0)
    dts = torch.empty(n, dtype=torch.float64, device="cuda")
    als = torch.empty((n, 6), dtype=torch.float64, device="cuda")
    st = torch.empty((n, 3, 4, 48, 48), dtype=torch.float64, device="cuda")
    assert s.run_save(U, n, st, dts, als) == n
    V = _dev(torch, U0)
    k, _, d2, a2 = s.run(V, n, record=True)
    assert k == n and torch.equal(U, V) and torch.equal(dts, d2)
    assert torch.equal(als.reshape(n, 2, 3).transpose(1, 2), a2)  # run() returns [step][stage][ax, ay]
    o = oracle_mod.Oracle(prm)
    W = U0.copy()
    dth = dts.cpu().numpy()
    alh = als.cpu().numpy().reshape(-1, 2, 3).transpose(0, 2, 1)
    U1 = torch.empty_like(V)
    U2 = torch.empty_like(V)
    for i in range(n):
        assert np.array_equal(st[i, 0].cpu().numpy(), W), i
        s.step_save(_dev(torch, W), dth[i], alh[i], U1, U2)
        assert torch.equal(st[i, 1], U1) and torch.equal(st[i, 2], U2), i
        W, _ = o.step(W, dth[i], alh[i])
    with pytest.raises(ValueError):
        s.run_save(U, n, st[:2], dts, als)
    with pytest.raises(hydro.HydroError):  # the state buffer may not be U itself
        s._check(s._lib.hydro_run_save(s._h, U.data_ptr(), 1, 0.0, None, None, None, U.data_ptr()),
                 "hydro_run_save")
    # stop at t_end after 3 steps: U holds the state after step 3
    t3 = float(dth[:3].sum())
    U = _dev(torch, U0)
    st.zero_()
    assert s.run_save(U, n, st, dts, als, t_end=t3) == 3
    assert torch.equal(U, st[3, 0])


def test_rollout_keeping_all_states_equals_checkpointed(torch, hydro):
    """ckpt_every=None (no replay) gives the checkpointed rollout's gradient bit
    for bit: the replay reproduces the forward's stage states exactly."""
    from paper_1507_08549_amd.autograd import rollout
    n, K, steps = 48, 8, 17
    prm = inputs.kh_sine_params(n)
    a_np = inputs.kh_sine_amplitudes(K, seed=5) * 20.0
    s = hydro.Solver(prm)
    grads = []
    for ck in (None, 5, 17):
        a = torch.tensor(a_np, dtype=torch.float64, device="cuda", requires_grad=True)
        UN = rollout(inputs.kh_sine_state(a, prm), s, steps, ckpt_every=ck)
        (g,) = torch.autograd.grad(_objective(torch, UN, prm), a)
        grads.append(g)
    assert torch.equal(grads[0], grads[1]) and torch.equal(grads[0], grads[2])


def test_checkpointed_rollout_backward_twice(torch, hydro):
    """The forward pass of a checkpointed rollout leaves the last segment's
    stage states for the backward pass (no replay of that segment); a second
    backward pass through the same graph replays every segment and gives the
    same gradient bit for bit, as does the rollout keeping every state."""
    from paper_1507_08549_amd.autograd import rollout
    n, K, steps = 40, 8, 13
    prm = inputs.kh_sine_params(n)
    a_np = inputs.kh_sine_amplitudes(K, seed=5) * 20.0
    s = hydro.Solver(prm)
    a = torch.tensor(a_np, dtype=torch.float64, device="cuda", requires_grad=True)
    J = _objective(torch, rollout(inputs.kh_sine_state(a, prm), s, steps, ckpt_every=5), prm)
    (g1,) = torch.autograd.grad(J, a, retain_graph=True)
    (g2,) = torch.autograd.grad(J, a)
    b = torch.tensor(a_np, dtype=torch.float64, device="cuda", requires_grad=True)
    (g0,) = torch.autograd.grad(
        _objective(torch, rollout(inputs.kh_sine_state(b, prm), s, steps, ckpt_every=None), prm), b)
    assert torch.equal(g1, g2) and torch.equal(g1, g0)


def test_adjoint_scratch_is_allocated_by_the_first_adjoint_call(torch, hydro):
    """A context holds two state-sized buffers; the first hydro_step_vjp_saved
    call adds three (stage adjoints, partial sum), the first hydro_step_vjp two
    more (recomputed stage states), later calls none; the results equal those
    of a context whose scratch was already there."""
    n = 1024
    prm, U0 = inputs.kelvin_helmholtz(n)
    state = 4 * n * n * 8
    rng = np.random.default_rng(4)
    U, lam = _dev(torch, U0), _dev(torch, rng.standard_normal(U0.shape))
    U1, U2, Un = torch.empty_like(U), torch.empty_like(U), torch.empty_like(U)
    out_a, out_b = torch.empty_like(U), torch.empty_like(U)
    free = lambda: (torch.cuda.synchronize(), torch.cuda.mem_get_info()[0])[1]
    f0 = free()
    s = hydro.Solver(prm)
    f1 = free()
    print(f"ADJ scratch: create {(f0 - f1) / state:.2f} states", flush=True)
    assert 1.9 * state <= f0 - f1 <= 2.3 * state
    dt = 0.2 * s.cfl(U)
    al = np.array([[3.0, 2.5], [3.1, 2.6], [3.2, 2.7]])
    s.step_save(U, dt, al, U1, U2, out=Un)
    f2 = free()
    s.step_vjp_saved(U, U1, U2, dt, al, lam, out=out_a)
    f3 = free()
    s.step_vjp(U, dt, al, lam, out=out_b)
    f4 = free()
    s.step_vjp_saved(U, U1, U2, dt, al, lam, out=out_a)
    s.step_vjp(U, dt, al, lam, out=out_b)
    f5 = free()
    print(f"ADJ scratch: first saved-state adjoint {(f2 - f3) / state:.2f}, "
          f"first recomputing adjoint {(f3 - f4) / state:.2f}, later {(f4 - f5) / state:.2f} states", flush=True)
    assert 2.7 * state <= f2 - f3 <= 3.3 * state
    assert 1.9 * state <= f3 - f4 <= 2.3 * state
    assert abs(f4 - f5) < 0.1 * state
    assert torch.equal(out_a, out_b)
    s.close()
