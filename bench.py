#!/usr/bin/env python3
"""Throughput of the WENO5 / global-LF / SSP-RK3 hot path on one MI355X.

Workload: the periodic shear layer (Kelvin-Helmholtz) on 512 x 512 cells,
gamma = 5/3, CFL 0.5, seeded v_y noise; one "step" is one full SSP-RK3 step
(three fused stage kernels: ghost fill, primitives, LF split, WENO5 in x and
y, divergence and sources, stage combination, LF/CFL max-reduction) with the
CFL time step computed on the device.  The state is resident in HBM before
the timed region starts.

Reported (one JSON line): FP64 cell-updates/s (the value), the FP32-bulk
form's rate and its relative L1 density error against the FP64 oracle, the
roofline of the stage kernel, the oracle's own rate on the host cores, and the
adjoint workload (sine-mode shear layer, 1024^2, 500 steps: backward/forward
time ratio in FP64 and FP32 keeping every state, and with checkpoints every
50 steps; central-difference check; FP32-vs-FP64 gradient error), and the potential solver on the polytrope
density (1024^2, red-black over-relaxation to the relative change 1e-8), the
level-set flame front (1025^2 corners: advection step and re-distancing), the
characteristic-wise reconstruction on the same shear layer (rate, and a few
steps against the oracle bit for bit), the step at 1024^2, 2048^2 and 4096^2
(states beyond the last-level cache), and two achievable-peak probes (FP64 fma
rate, device copy).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one stage per cell (FP64 operations of the method, an
# fma counted as 2 flops, a division or square root as 1): primitives and
# split fluxes at the point for x and y (2 x 41), 8 WENO5 reconstructions
# (8 x 66) plus the face sums (4) for the x face and the same for the y face
# (2 x 532), divergence, sources, stage combination, output primitives and
# the maxima (64).  See the design notes for the itemised count.
FLOPS_PER_CELL_STAGE = 2 * 41 + 2 * (8 * 66 + 4) + 64
# Algorithmic HBM bytes of one step per cell: stage 1 reads U^n and writes U1;
# stages 2 and 3 read U^n and their input and write their output (FP64 x 4).
BYTES_PER_CELL_STEP = 32 * (2 + 3 + 3)
PEAK_FP64_VALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic bytes of one red-black iteration per cell: rho once, the
# potential read twice (as a cell of its colour and as a neighbour of the
# other) and written once (FP64).
POISSON_BYTES_PER_CELL_ITER = 8 * 4


# HBM traffic of one stage-kernel launch on this workload, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by the factors a 256 MiB device
# copy gives (x2.0 for FETCH, x1.0 for WRITE); the summary, with the commands,
# is under profiles/.  It holds for the kernel sources with this digest only:
# after any change to them the figure is reported as null until re-measured.
STAGE_TRAFFIC = {
    "sources": ["paper_1507_08549_amd/csrc/stage_kernel.hpp", "paper_1507_08549_amd/csrc/ieee.hpp",
                "paper_1507_08549_amd/csrc/stage_fp64.hip", "paper_1507_08549_amd/csrc/hydro_internal.hpp"],
    "sha256": "391f199656abe7698864bd73113063a5ae8ae9e81bd68b19ab537271b74a946f",
    "n": 512,
    "bytes_per_launch": (15.192 + 8.489) * 1e6,
    # SQ_INSTS_VALU of the same launch (wavefront instructions), same digest
    "valu_insts_per_launch": 6804486,
}
# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles per
# SIMD at 2.4 GHz (FP64 add, mul and fma issue at that rate).
PEAK_VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4


def stage_measured(n, key):
    """A counter figure of the stage kernel (HBM bytes or VALU instructions per
    launch), or None once its sources or the grid differ from the measured."""
    import hashlib
    h = hashlib.sha256()
    for f in STAGE_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != STAGE_TRAFFIC["sha256"] or n != STAGE_TRAFFIC["n"]:
        return None
    return STAGE_TRAFFIC[key]


def stage_traffic(n):
    return stage_measured(n, "bytes_per_launch")


def host_cpu():
    """Model name and logical CPU count of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_run(torch, solver, U, steps):
    """Time `steps` steps (device-side CFL) with HIP events on the solver's stream."""
    st = solver.stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    t0 = time.perf_counter()
    solver.run(U, steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def adjoint_leg(torch, hydro, inputs, n, steps, ckpt, precision, a_np, sched=None):
    """Gradient of the final y-kinetic energy of the sine-mode shear layer with
    respect to its mode amplitudes, by the hand-written adjoint (rollout keeping
    every state when ckpt is None, else checkpointed every ckpt steps).
    Returns (solver, J, grad, forward seconds, backward seconds, schedule)."""
    from paper_1507_08549_amd.autograd import rollout
    prm = inputs.kh_sine_params(n)
    s = hydro.Solver(prm, precision=precision)
    dxdy = 1.0 / (n * n)

    def once(nsteps):
        a = torch.tensor(a_np, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        UN = rollout(inputs.kh_sine_state(a, prm), s, nsteps, ckpt)
        J = (0.5 * UN[2] * UN[2] / UN[0]).sum() * dxdy
        J.item()
        t1 = time.perf_counter()
        (g,) = torch.autograd.grad(J, a)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return J.item(), g.cpu().numpy(), t1 - t0, t2 - t1

    once(min(steps, 2 * (ckpt or 50)))  # warm-up (allocations, code objects)
    J, g, tf, tb = once(steps)
    if sched is None:  # the schedule of this rollout (bit-identical replay)
        U = inputs.kh_sine_state(torch.tensor(a_np, dtype=torch.float64, device="cuda"), prm).contiguous()
        _, _, dts, als = s.run(U, steps, record=True)
        sched = (dts.cpu().numpy(), als.cpu().numpy())
    return s, J, g, tf, tb, sched


def fd_check(torch, inputs, s, a_np, sched, comps, h=1e-7):
    """Central differences of J along mode amplitudes, replaying the schedule."""
    prm = s.params
    n = prm["nx"]
    dts, als = sched

    def J_of(av):
        U = inputs.kh_sine_state(torch.tensor(av, dtype=torch.float64, device="cuda"), prm).contiguous()
        for dt, al in zip(dts, als):
            s.step(U, float(dt), alpha=al)
        return ((0.5 * U[2] * U[2] / U[0]).sum() / (n * n)).item()

    out = []
    for k in comps:
        e = np.zeros_like(a_np)
        e[k] = h
        out.append((J_of(a_np + e) - J_of(a_np - e)) / (2 * h))
    return np.array(out)


PROBE_LIB = os.path.join(ROOT, "paper_1507_08549_amd", "libhydro_probe.so")


def fma_probe_rate(torch, iters=20000):
    """Achievable FP64 fma rate (flop/s) of the current device, from the
    measurement library's probe kernel (csrc/probe.h), on torch's current
    stream."""
    import ctypes
    if not os.path.exists(PROBE_LIB):
        raise RuntimeError(f"{PROBE_LIB} is missing: build it with paper_1507_08549_amd.build.build()")
    lib = ctypes.CDLL(PROBE_LIB)
    lib.hydro_probe_fma_rate.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.hydro_probe_fma_rate.restype = ctypes.c_int
    r = ctypes.c_double()
    rc = lib.hydro_probe_fma_rate(int(iters), torch.cuda.current_stream().cuda_stream, ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"hydro_probe_fma_rate failed ({rc})")
    return r.value


def probes(torch):
    """Achievable-peak references: the FP64 fma rate (probe kernel) and a 1 GiB
    device-to-device copy (read + written bytes per second)."""
    fma = fma_probe_rate(torch, 20000)
    nel = (1 << 30) // 8
    src = torch.ones(nel, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 5 * 2 * (1 << 30) / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    out = {"fp64_fma_tflops": fma / 1e12, "fp64_fma_frac_of_peak": fma / 1e12 / PEAK_FP64_VALU_TFLOPS,
           "copy_gbs": gbs, "copy_frac_of_peak": gbs / PEAK_HBM_GBS}
    log(f"probes: fp64 fma {out['fp64_fma_tflops']:.1f} TFLOP/s, copy {gbs:.0f} GB/s")
    return out


def sweep_leg(torch, hydro, inputs, sizes, steps):
    """The FP64 step at sizes whose states no longer fit in the 256 MB
    last-level cache: cell-updates/s and the algorithmic HBM rate."""
    out = []
    for n in sizes:
        prm, U0 = inputs.kelvin_helmholtz(n, seed=2)
        s = hydro.Solver(prm)
        U = torch.tensor(U0, dtype=torch.float64, device="cuda")
        del U0
        s.run(U, 10)
        t, _ = timed_run(torch, s, U, steps)
        r = {"n": n, "steps": steps, "ms_per_step": t * 1e3 / steps,
             "cell_updates_per_s": n * n * steps / t,
             "hbm_gbs_algorithmic": BYTES_PER_CELL_STEP * n * n * steps / t / 1e9,
             "state_mb": 32 * n * n / 1e6}
        r["hbm_frac"] = r["hbm_gbs_algorithmic"] / PEAK_HBM_GBS
        log(f"sweep {n}^2: {r['cell_updates_per_s']:.3e} cell-updates/s, {r['hbm_gbs_algorithmic']:.0f} GB/s")
        out.append(r)
        s.close()
        del U
        torch.cuda.empty_cache()
    return out


def charwise_leg(torch, hydro, inputs, n, steps, cpu_steps):
    """The characteristic-wise reconstruction (Roe-averaged eigenvectors at
    every face, the "WENO-Roe" option of Sect. 2.1) on the same shear layer,
    FP64: cell-updates/s; on the host, the oracle's characteristic path for a
    few steps from the same start, compared bit for bit."""
    prm, U0 = inputs.kelvin_helmholtz(n, seed=2)
    prm = dict(prm, recon=hydro.CHARACTERISTIC)
    s = hydro.Solver(prm)
    U = torch.tensor(U0, dtype=torch.float64, device="cuda")
    s.run(U, 10)
    t, _ = timed_run(torch, s, U, steps)
    res = {"workload": f"kelvin_helmholtz_{n}x{n}", "reconstruction": "characteristic",
           "precision": "fp64", "steps": steps, "ms_per_step": t * 1e3 / steps,
           "cell_updates_per_s": n * n * steps / t, "kernel": "stage_kernel<double,16,16,true,true>"}
    if cpu_steps > 0:
        import oracle
        c0 = time.perf_counter()
        ref, _, _, _ = oracle.Oracle(prm).run(U0, cpu_steps)
        ct = time.perf_counter() - c0
        Uc = torch.tensor(U0, dtype=torch.float64, device="cuda")
        s.run(Uc, cpu_steps)
        res["oracle_cell_updates_per_s"] = n * n * cpu_steps / ct
        res["oracle_steps"] = cpu_steps
        res["bitwise_equal_oracle"] = bool(np.array_equal(Uc.cpu().numpy(), ref))
    log(f"characteristic: {res['cell_updates_per_s']:.3e} cell-updates/s"
        + (f", oracle {res['oracle_cell_updates_per_s']:.3e} over {cpu_steps} steps, bitwise "
           f"{res['bitwise_equal_oracle']}" if cpu_steps > 0 else ""))
    s.close()
    return res


def configs_leg(torch, hydro, inputs):
    """The other workloads at their full lengths, FP64 and FP32-bulk: rates, the
    FP32 form's relative L1 density error against the FP64 path (which matches
    the oracle bit for bit on every prefix the tests check), and the
    polytrope's equilibrium drift (max |v| / c_center and the L1 density change
    after 1000 steps; no exact value exists, the scheme is not well balanced)."""
    cases = [("kelvin_helmholtz_512x512_2000steps", lambda: inputs.kelvin_helmholtz(512, seed=2) + (None,), 2000),
             ("rayleigh_taylor_256x1024_5000steps", lambda: inputs.rayleigh_taylor() + (None,), 5000),
             ("polytrope_1024x1024_1000steps", lambda: inputs.polytrope(1024), 1000)]
    out = []
    for name, make, steps in cases:
        prm, U0, grav = make()
        g = None if grav is None else torch.tensor(grav, dtype=torch.float64, device="cuda")
        res = {"workload": name}
        fin = {}
        for prec, key in ((hydro.FP64, "fp64"), (hydro.FP32_BULK, "fp32")):
            s = hydro.Solver(prm, gravity=g, precision=prec)
            U = torch.tensor(U0, dtype=torch.float64, device="cuda")
            t, _ = timed_run(torch, s, U, steps)
            res[f"{key}_cell_updates_per_s"] = prm["nx"] * prm["ny"] * steps / t
            fin[key] = U
            s.close()
        d = (fin["fp32"][0] - fin["fp64"][0]).abs().sum() / fin["fp64"][0].abs().sum()
        res["fp32_l1_rel_density_err_vs_fp64"] = float(d)
        if grav is not None:
            U = fin["fp64"]
            rho0 = torch.tensor(U0[0], dtype=torch.float64, device="cuda")
            vmag = torch.sqrt(U[1] ** 2 + U[2] ** 2) / U[0]
            dense = rho0 > 1e-3
            res["drift_l1_rel_density"] = float((U[0] - rho0).abs().sum() / rho0.abs().sum())
            res["drift_max_speed_over_c_center_dense"] = float(vmag[dense].max() / math.sqrt(4.0 / 3.0))
        log(f"config {name}: fp64 {res['fp64_cell_updates_per_s']:.3e}, fp32 {res['fp32_cell_updates_per_s']:.3e} "
            f"cell-updates/s, fp32 L1 err {res['fp32_l1_rel_density_err_vs_fp64']:.2e}")
        out.append(res)
    return out


def poisson_leg(torch, hydro, inputs, n, cpu_iters):
    """Potential of the n = 3 polytrope's density from a zero start to the
    relative change 1e-8 with the near-optimal over-relaxation factor."""
    import math
    prm, U0, _ = inputs.polytrope(n)
    L = prm["xhi"]
    rho_np = np.ascontiguousarray(U0[0])
    dr = L / n
    r = (np.arange(n) + 0.5) * dr
    mass = 2.0 * float((2.0 * math.pi * r[None, :] * rho_np * dr * dr).sum())
    omega = 2.0 / (1.0 + math.sin(math.pi / n))
    qprm = inputs.make_params(n, n, 0.0, L, 0.0, L, prm["bc"], prm["gamma"], geometry=inputs.CYLINDRICAL)
    s = hydro.Solver(qprm)
    rho = torch.tensor(rho_np, dtype=torch.float64, device="cuda")
    phi = torch.zeros_like(rho)
    s.poisson(rho, phi, 1.0, mass, omega=omega, tol=1e-8, max_iter=50)  # warm-up
    phi.zero_()
    st = s.stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    t0 = time.perf_counter()
    iters, change = s.poisson(rho, phi, 1.0, mass, omega=omega, tol=1e-8, max_iter=200000)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t = e0.elapsed_time(e1) / 1e3
    out = {"workload": f"polytrope_density_{n}x{n}_zero_start_tol1e-8", "omega": omega,
           "iterations": iters, "last_change": change, "ms": t * 1e3, "wall_ms": wall * 1e3,
           "cell_iterations_per_s": n * n * iters / t,
           "us_per_iteration": t * 1e6 / iters,
           "hbm_gbs_algorithmic": POISSON_BYTES_PER_CELL_ITER * n * n * iters / t / 1e9}
    out["hbm_frac"] = out["hbm_gbs_algorithmic"] / PEAK_HBM_GBS
    log(f"poisson: {iters} iterations in {t * 1e3:.1f} ms ({out['us_per_iteration']:.2f} us/iteration, "
        f"{out['hbm_gbs_algorithmic']:.0f} GB/s algorithmic)")
    if cpu_iters > 0:
        import oracle
        c0 = time.perf_counter()
        ref, _, _ = oracle.poisson(rho_np, L, L, 1.0, mass, omega=omega, tol=0.0, max_iter=cpu_iters)
        ct = time.perf_counter() - c0
        phi.zero_()
        s.poisson(rho, phi, 1.0, mass, omega=omega, tol=0.0, max_iter=cpu_iters)
        out["cpu_oracle"] = {"cell_iterations_per_s": n * n * cpu_iters / ct, "cores": 1,
                             "sample": f"{cpu_iters} iterations, {ct:.1f} s",
                             "fp64_bitwise_equal": bool(np.array_equal(phi.cpu().numpy(), ref))}
    s.close()
    return out


def levelset_leg(torch, hydro, inputs, n, steps, cpu):
    """Level-set flame front on (n+1)^2 corners: `steps` rounds of one SSP-RK3
    advection step and one re-distancing, each timed with HIP events."""
    prm, S0, vel_np, s_f = inputs.flame_front(n)
    s = hydro.Solver(prm)
    S = torch.tensor(S0, dtype=torch.float64, device="cuda")
    vel = torch.tensor(vel_np, dtype=torch.float64, device="cuda")
    dt = 0.5 / n / (float(np.abs(vel_np).max()) + s_f)
    st = s.stream
    for _ in range(2):
        s.ls_step(S, vel, s_f, dt)
        s.ls_redistance(S)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_step = t_red = 0.0
    npts = 0
    for _ in range(steps):
        ev[0].record(st)
        s.ls_step(S, vel, s_f, dt)
        ev[1].record(st)
        npts = s.ls_redistance(S)
        ev[2].record(st)
        torch.cuda.synchronize()
        t_step += ev[0].elapsed_time(ev[1]) / 1e3
        t_red += ev[1].elapsed_time(ev[2]) / 1e3
    nc = (n + 1) * (n + 1)
    out = {"workload": f"flame_front_{n}x{n}_cells_{n + 1}x{n + 1}_corners", "steps": steps,
           "step_us": t_step * 1e6 / steps, "redistance_us": t_red * 1e6 / steps,
           "front_points": npts,
           "corner_updates_per_s": nc * steps / t_step,
           "distance_pairs_per_s_bruteforce_equiv": float(nc) * npts * steps / t_red}
    log(f"levelset: step {out['step_us']:.1f} us, redistance {out['redistance_us']:.1f} us "
        f"({npts} front points)")
    if cpu:
        import oracle
        ls = oracle.LevelSet(prm)
        c0 = time.perf_counter()
        ls.step(S0, vel_np, s_f, dt)
        ct = time.perf_counter() - c0
        out["cpu_oracle"] = {"corner_updates_per_s": nc / ct, "cores": 1,
                             "sample": f"one advection step at full size, {ct:.2f} s"}
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=512, help="grid size (n x n)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of K steps (the first is the value; all give the median)")
    ap.add_argument("--cpu-steps", type=int, default=100,
                    help="oracle steps timed for the CPU baseline (0: skip)")
    ap.add_argument("--only-fp64", action="store_true", help="skip the FP32-bulk leg")
    ap.add_argument("--char-steps", type=int, default=400,
                    help="steps of the characteristic-reconstruction leg (0: skip)")
    ap.add_argument("--char-cpu-steps", type=int, default=3,
                    help="oracle steps of that leg compared bit for bit")
    ap.add_argument("--adj-n", type=int, default=1024, help="adjoint workload grid (n x n; 0: skip)")
    ap.add_argument("--adj-steps", type=int, default=500)
    ap.add_argument("--adj-ckpt", type=int, default=50,
                    help="checkpoint interval of the checkpointed adjoint figure (the headline keeps all states)")
    ap.add_argument("--poisson-n", type=int, default=1024,
                    help="potential-solver workload grid (n x n; 0: skip)")
    ap.add_argument("--poisson-cpu-iters", type=int, default=200)
    ap.add_argument("--ls-n", type=int, default=1024, help="level-set workload cells per side (0: skip)")
    ap.add_argument("--ls-steps", type=int, default=20)
    ap.add_argument("--sweep", type=str, default="1024,2048,4096",
                    help="grid sizes of the out-of-cache sweep (comma separated; empty: skip)")
    ap.add_argument("--sweep-steps", type=int, default=200)
    ap.add_argument("--no-probes", action="store_true", help="skip the fma-rate and copy probes")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the full-length runs of the other workloads (shear layer 2000 steps, "
                         "heavy-over-light layer 5000, polytrope 1000)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB three times (a known-size "
                         "kernel for calibrating the profiler's HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU only; --gpus must be 1 "
              "(the multi-GPU decomposition is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1507_08549_amd import hydro, inputs

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    n = args.n
    prm, U0 = inputs.kelvin_helmholtz(n, seed=2)
    ncell = n * n

    # ---- FP64 (the value)
    s64 = hydro.Solver(prm, precision=hydro.FP64)
    U = torch.tensor(U0, dtype=torch.float64, device="cuda")
    s64.run(U, args.warmup)
    t64, wall64 = timed_run(torch, s64, U, args.steps)
    v64 = ncell * args.steps / t64
    log(f"fp64: {args.steps} steps in {t64 * 1e3:.2f} ms (wall {wall64 * 1e3:.2f}) -> {v64:.4e} cell-updates/s")
    # the same K steps timed again (the flow continues), for the spread over runs
    reps = [v64]
    for _ in range(max(args.repeats, 1) - 1):
        t, _ = timed_run(torch, s64, U, args.steps)
        reps.append(ncell * args.steps / t)
    repeats = {"runs": len(reps), "median": float(np.median(reps)), "min": min(reps), "max": max(reps)}
    if len(reps) > 1:
        log(f"fp64 over {len(reps)} runs of {args.steps} steps: median {repeats['median']:.4e}, "
            f"min {repeats['min']:.4e}, max {repeats['max']:.4e}")

    # stage-kernel average duration: 3 stage launches per step (plus three tiny
    # set-up kernels per call, included, so the estimate is conservative)
    stage_s = t64 / (3 * args.steps)
    # the binding roof as instruction issue: measured VALU instructions per
    # launch over the launch time, against the issue peak
    insts = stage_measured(n, "valu_insts_per_launch")
    issue = None if insts is None else {
        "valu_wave_insts_per_launch": insts, "achieved_per_s": insts / stage_s,
        "peak_per_s": PEAK_VALU_WAVE_INSTS_PER_S, "frac": insts / stage_s / PEAK_VALU_WAVE_INSTS_PER_S}
    flops_launch = FLOPS_PER_CELL_STAGE * ncell
    achieved_tf = flops_launch / stage_s / 1e12
    hbm_gbs = BYTES_PER_CELL_STEP * ncell / 3 / stage_s / 1e9

    # ---- FP32 bulk
    fp32 = None
    if not args.only_fp64:
        s32 = hydro.Solver(prm, precision=hydro.FP32_BULK)
        U32 = torch.tensor(U0, dtype=torch.float64, device="cuda")
        s32.run(U32, args.warmup)
        t32, _ = timed_run(torch, s32, U32, args.steps)
        fp32 = {"value": ncell * args.steps / t32, "ms_per_step": t32 * 1e3 / args.steps}
        log(f"fp32-bulk: {fp32['value']:.4e} cell-updates/s")

    # ---- oracle on the host (bounded sample), and the errors it pins
    cpu = None
    if args.cpu_steps > 0:
        import oracle
        o = oracle.Oracle(prm)
        c0 = time.perf_counter()
        ref, _, _, _ = o.run(U0, args.cpu_steps)
        ct = time.perf_counter() - c0
        cpu = {"value": ncell * args.cpu_steps / ct, "unit": "cell-updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{args.cpu_steps} SSP-RK3 steps of the same {n}x{n} shear layer, "
                         f"single-threaded C oracle, {ct:.1f} s"}
        cpu["host"] = host_cpu()
        log(f"oracle: {cpu['value']:.4e} cell-updates/s ({ct:.1f} s)")
        Uc = torch.tensor(U0, dtype=torch.float64, device="cuda")
        s64.run(Uc, args.cpu_steps)
        g64 = Uc.cpu().numpy()
        cpu["fp64_bitwise_equal"] = bool(np.array_equal(g64, ref))
        if fp32 is not None:
            U32 = torch.tensor(U0, dtype=torch.float64, device="cuda")
            s32.run(U32, args.cpu_steps)
            g32 = U32.cpu().numpy()
            fp32["l1_rel_density_err_vs_oracle"] = float(np.abs(g32[0] - ref[0]).sum() / np.abs(ref[0]).sum())
            fp32["err_steps"] = args.cpu_steps

    # ---- adjoint: sine-mode shear layer, gradient of the final y-kinetic energy
    adj = None
    if args.adj_n > 0:
        a_np = inputs.kh_sine_amplitudes()
        # headline: every state kept (3 x 500 states of 32 MiB at 1024^2), no replay
        s64a, J64, g64, tf64, tb64, sched = adjoint_leg(torch, hydro, inputs, args.adj_n, args.adj_steps,
                                                       None, hydro.FP64, a_np)
        _, J32, g32, tf32, tb32, _ = adjoint_leg(torch, hydro, inputs, args.adj_n, args.adj_steps,
                                                 None, hydro.FP32_BULK, a_np, sched)
        # the same gradient with checkpoints (stage states recomputed per segment)
        _, _, g64c, tf64c, tb64c, _ = adjoint_leg(torch, hydro, inputs, args.adj_n, args.adj_steps,
                                                  args.adj_ckpt, hydro.FP64, a_np, sched)
        _, _, _, tf32c, tb32c, _ = adjoint_leg(torch, hydro, inputs, args.adj_n, args.adj_steps,
                                               args.adj_ckpt, hydro.FP32_BULK, a_np, sched)
        comps = [0, 17, 63]
        fd = fd_check(torch, inputs, s64a, a_np, sched, comps)
        fd_err = float(np.max(np.abs(fd - g64[comps]) / np.abs(g64).max()))
        adj = {"workload": f"kh_sine_{args.adj_n}x{args.adj_n}_{args.adj_steps}steps",
               "J": J64,
               "states_kept_gb": 3 * args.adj_steps * 32 * args.adj_n * args.adj_n / 1e9,
               "fwd_ms_fp64": tf64 * 1e3, "bwd_ms_fp64": tb64 * 1e3, "ratio_fp64": tb64 / tf64,
               "fwd_ms_fp32": tf32 * 1e3, "bwd_ms_fp32": tb32 * 1e3, "ratio_fp32": tb32 / tf32,
               "ckpt_every": args.adj_ckpt,
               "ratio_fp64_ckpt": tb64c / tf64c, "ratio_fp32_ckpt": tb32c / tf32c,
               "ckpt_grad_bitwise_equal": bool(np.array_equal(g64c, g64)),
               "fd_components": comps, "fd_rel_err_fp64": fd_err,
               "grad_rel_err_fp32_vs_fp64": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))}
        log(f"adjoint: fp64 ratio {adj['ratio_fp64']:.2f} (fwd {tf64 * 1e3:.1f} ms, bwd {tb64 * 1e3:.1f} ms), "
            f"fp32 ratio {adj['ratio_fp32']:.2f}; checkpointed every {args.adj_ckpt}: "
            f"{adj['ratio_fp64_ckpt']:.2f} / {adj['ratio_fp32_ckpt']:.2f}; FD rel err {fd_err:.2e}, "
            f"fp32 grad rel err {adj['grad_rel_err_fp32_vs_fp64']:.2e}")

    prb = None if args.no_probes else probes(torch)
    sweep = None
    if args.sweep:
        sweep = sweep_leg(torch, hydro, inputs, [int(v) for v in args.sweep.split(",") if v], args.sweep_steps)

    cfgs = None if args.no_configs else configs_leg(torch, hydro, inputs)

    pois = None
    if args.poisson_n > 0:
        pois = poisson_leg(torch, hydro, inputs, args.poisson_n,
                           args.poisson_cpu_iters if args.cpu_steps > 0 else 0)

    chw = None
    if args.char_steps > 0:
        chw = charwise_leg(torch, hydro, inputs, n, args.char_steps,
                           args.char_cpu_steps if args.cpu_steps > 0 else 0)

    lset = None
    if args.ls_n > 0:
        lset = levelset_leg(torch, hydro, inputs, args.ls_n, args.ls_steps, args.cpu_steps > 0)

    out = {
        "metric": "cell-updates/sec per RK3 step FP64 vs FP32 at stated L1 err; adjoint/fwd ratio",
        "value": v64,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t64 * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"kelvin_helmholtz_{n}x{n}", "nx": n, "ny": n, "gamma": 5.0 / 3.0,
                   "cfl": 0.5, "bc": "periodic", "seed": 2, "precision": "fp64"},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP64_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tf / PEAK_FP64_VALU_TFLOPS,
                     "traffic": stage_traffic(n), "traffic_unit": "bytes per launch",
                     "algorithmic_bytes_per_launch": BYTES_PER_CELL_STEP * ncell / 3,
                     "kernel": "stage_kernel<double,16,16>",
                     "avg_launch_us": stage_s * 1e6, "hbm_gbs_algorithmic": hbm_gbs,
                     "hbm_frac": hbm_gbs / PEAK_HBM_GBS, "issue": issue},
        "repeats": repeats,
        "cpu_baseline": cpu,
        "fp32_bulk": fp32,
        "adjoint": adj,
        "configs": cfgs,
        "probes": prb,
        "sweep": sweep,
        "poisson": pois,
        "levelset": lset,
        "characteristic": chw,
    }
    print(json.dumps(out), flush=True)

    if args.copy_probe > 0:
        nel = args.copy_probe * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written per copy, 3 copies")


if __name__ == "__main__":
    main()
