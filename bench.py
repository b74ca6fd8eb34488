#!/usr/bin/env python3
"""Throughput of the WENO5 / global-LF / SSP-RK3 hot path on one MI355X.

Workload (the value): the n = 3 polytrope in cylindrical (r, z) geometry on
1024 x 1024 cells, gamma = 4/3, CFL 0.5, fixed gravity field from the
enclosed mass, atmosphere floors at rho = 1e-8, seeded 1e-3 density noise:
its 1000 SSP-RK3 steps from the initial state.  One step is three fused stage
kernels (ghost fill, primitives, LF split, WENO5 in x and y, divergence,
gravity and geometric sources, stage combination, floors, LF/CFL
max-reduction) with the CFL time step computed on the device.  The state and
the gravity field are resident in HBM before the timed region starts.

Reported (one JSON line): FP64 cell-updates/s (the value) with the final
state's digest checked against the oracle's; the stage kernel's roofline
(per-launch time from the difference of a K-step run and an empty run, both
timed with HIP events on the solver's stream); the FP32-bulk form's rate and
relative L1 density error against the oracle; the oracle's own rate on the
host (one thread and all cores); and further legs: the periodic shear layer
(512^2) with its own roofline, the other workloads at full length, the
adjoint workload (sine-mode shear layer, 1024^2, 500 steps: backward/forward
ratio, FP32-bulk with checkpoints every 50 steps as the headline figure,
central differences of all 64 mode amplitudes), the potential solver, the
level-set flame front, the characteristic-wise reconstruction, the step at
2048^2 and 4096^2, and two achievable-peak probes (FP64 fma rate, device
copy).
"""
from __future__ import annotations

import argparse
import hashlib
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
# (2 x 532), divergence, uniform or field gravity, stage combination, output
# primitives and the maxima (64).  See the design notes for the itemised count.
FLOPS_PER_CELL_STAGE = 2 * 41 + 2 * (8 * 66 + 4) + 64
# The polytrope adds the geometric sources of the cylindrical form (the cell's
# primitives 12, its radius and 1/r 3, four source terms 12) and the pressure
# floor's primitives of the new state (12).
FLOPS_PER_CELL_STAGE_CYL_FLOORS = FLOPS_PER_CELL_STAGE + 27 + 12
# Algorithmic HBM bytes of one step per cell: stage 1 reads U^n and writes U1;
# stages 2 and 3 read U^n and their input and write their output (FP64 x 4);
# with a gravity field each stage also reads (g_x, g_y) (2 x 8 B x 3).
BYTES_PER_CELL_STEP = 32 * (2 + 3 + 3)
BYTES_PER_CELL_STEP_FIELD = BYTES_PER_CELL_STEP + 3 * 16
PEAK_FP64_VALU_TFLOPS = 78.6
# Published dense FP32 vector peak; it counts packed FP32 instructions, which
# this build does not use (unpacked FP32 issues at the FP64 rate).
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# Algorithmic bytes of one red-black iteration per cell: rho once, the
# potential read twice (as a cell of its colour and as a neighbour of the
# other) and written once (FP64): the count of a solver with one sweep per
# launch.  The temporally blocked kernel moves less (measured below).
POISSON_BYTES_PER_CELL_ITER = 8 * 4
# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles per
# SIMD at 2.4 GHz (FP64 add, mul and fma issue at that rate).
PEAK_VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4

STAGE_SOURCES = ["paper_1507_08549_amd/csrc/stage_kernel.hpp", "paper_1507_08549_amd/csrc/ieee.hpp",
                 "paper_1507_08549_amd/csrc/stage_fp64.hip", "paper_1507_08549_amd/csrc/hydro_internal.hpp"]
# Counter figures of one FP64 stage-kernel launch per workload: HBM traffic
# from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by the factors
# a 256 MiB device copy gives (x2.0 for FETCH, x1.0 for WRITE), and
# SQ_INSTS_VALU (wavefront instructions).  The summaries, with the commands,
# are under profiles/.  They hold for the kernel sources with this digest only:
# after any change to them the figures are reported as null until re-measured.
STAGE_COUNTERS = {
    "sha256": "b8e97aa824861336a06b06ca0e362bcb623f8f1d5e53eebee7a797b44d27696c",
    "workloads": {
        "polytrope_1024x1024": {"bytes_per_launch": (36943.7 * 1.99974 + 33154.0) * 1024,
                                "valu_insts_per_launch": 24005834},
        "kelvin_helmholtz_512x512": {"bytes_per_launch": (7409.1 * 1.99974 + 8290.0) * 1024,
                                     "valu_insts_per_launch": 5793033},
    },
}
# The potential solver's launch (4 iterations): measured HBM bytes and VALU
# instructions (profiles/poisson_block_polytrope1024.md).
POISSON_COUNTERS = {"sources": ["paper_1507_08549_amd/csrc/poisson.hip"],
                    "sha256": "c48f737c8cdd706a942694d626cff0899aa68d4c680dc421ecbb8406d5215aa6", "iterations_per_launch": 4,
                    "bytes_per_launch": 18.63e6 + 8.27e6, "valu_insts_per_launch": 9065717,
                    "launch_us": 28.08}


def sources_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stage_measured(workload, key):
    """A counter figure of the FP64 stage kernel (HBM bytes or VALU instructions
    per launch) on a workload, or None once its sources differ from the
    measured ones or the workload was not measured."""
    w = STAGE_COUNTERS["workloads"].get(workload)
    if w is None or sources_digest(STAGE_SOURCES) != STAGE_COUNTERS["sha256"]:
        return None
    return w.get(key)


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


def run_overhead(torch, solver, U, reps=7):
    """Event time of a run of zero steps (the per-call set-up kernels and the
    final read-back), median of reps: subtracted from a K-step run it leaves
    the 3K stage launches."""
    return float(np.median([timed_run(torch, solver, U, 0)[0] for _ in range(reps)]))


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


def golden_state_digest(name, step):
    """The oracle's state digest of a workload at a checkpoint (tests/golden), or None."""
    path = os.path.join(ROOT, "tests", "golden", "full_length.json")
    try:
        with open(path) as f:
            w = json.load(f)["workloads"][name]
    except (OSError, KeyError, ValueError):
        return None
    for cp in w["checkpoints"]:
        if cp["step"] == step:
            return cp["state"]
    return None


def stage_roofline(torch, solver, U0d, steps, ncell, flops_cell, bytes_cell_step, workload, kernel):
    """Per-launch time of the FP64 stage kernel from K steps minus an empty run
    (both event-timed on the solver's stream), and the roofline it gives."""
    U = U0d.clone()
    t_k, _ = timed_run(torch, solver, U, steps)
    t_0 = run_overhead(torch, solver, U)
    stage_s = (t_k - t_0) / (3 * steps)
    achieved = flops_cell * ncell / stage_s / 1e12
    insts = stage_measured(workload, "valu_insts_per_launch")
    issue = None if insts is None else {
        "valu_wave_insts_per_launch": insts, "achieved_per_s": insts / stage_s,
        "peak_per_s": PEAK_VALU_WAVE_INSTS_PER_S, "frac": insts / stage_s / PEAK_VALU_WAVE_INSTS_PER_S}
    hbm = bytes_cell_step * ncell / 3 / stage_s / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VALU_TFLOPS,
            "traffic": stage_measured(workload, "bytes_per_launch"), "traffic_unit": "bytes per launch",
            "algorithmic_flops_per_launch": flops_cell * ncell,
            "algorithmic_bytes_per_launch": bytes_cell_step * ncell / 3,
            "kernel": kernel, "avg_launch_us": stage_s * 1e6,
            "timing": f"({steps} steps {t_k * 1e3:.3f} ms - empty run {t_0 * 1e3:.3f} ms) / {3 * steps} launches",
            "hbm_gbs_algorithmic": hbm, "hbm_frac": hbm / PEAK_HBM_GBS, "issue": issue}


def headline_leg(torch, hydro, inputs, args):
    """The polytrope's 1000 steps from its initial state, FP64 (timed K steps,
    repeated from the same start), the stage roofline, FP32-bulk beside it."""
    name = "polytrope_1024"
    prm, U0, grav = inputs.polytrope(1024)
    ncell = prm["nx"] * prm["ny"]
    g = torch.tensor(grav, dtype=torch.float64, device="cuda")
    U0d = torch.tensor(U0, dtype=torch.float64, device="cuda")
    s64 = hydro.Solver(prm, gravity=g, precision=hydro.FP64)
    U = U0d.clone()
    s64.run(U, args.warmup)  # warm-up on a copy: clocks, code objects
    runs = []
    final = None
    for r in range(max(args.repeats, 1)):
        U = U0d.clone()
        t, wall = timed_run(torch, s64, U, args.steps)
        runs.append(ncell * args.steps / t)
        if r == 0:
            t64, wall64 = t, wall
            final = U.cpu().numpy()
    v64 = runs[0]
    log(f"fp64: {args.steps} steps of the 1024^2 polytrope in {t64 * 1e3:.2f} ms (wall {wall64 * 1e3:.2f}) "
        f"-> {v64:.4e} cell-updates/s; over {len(runs)} runs median {np.median(runs):.4e}")
    want = golden_state_digest(name, args.steps)
    check = None if want is None else bool(digest(final) == want)
    roof = stage_roofline(torch, s64, U0d, args.steps, ncell, FLOPS_PER_CELL_STAGE_CYL_FLOORS,
                          BYTES_PER_CELL_STEP_FIELD, "polytrope_1024x1024",
                          "stage_kernel<double,16,16,true,false>")
    log(f"stage kernel: {roof['avg_launch_us']:.2f} us per launch, {roof['achieved']:.1f} TFLOP/s "
        f"({roof['frac']:.3f} of the FP64 peak)")
    fp32 = None
    if not args.only_fp64:
        s32 = hydro.Solver(prm, gravity=g, precision=hydro.FP32_BULK)
        U32 = U0d.clone()
        s32.run(U32, args.warmup)
        U32 = U0d.clone()
        t32, _ = timed_run(torch, s32, U32, args.steps)
        stage32 = (t32 - run_overhead(torch, s32, U0d.clone())) / (3 * args.steps)
        ach32 = FLOPS_PER_CELL_STAGE_CYL_FLOORS * ncell / stage32 / 1e12
        fp32 = {"value": ncell * args.steps / t32, "ms_per_step": t32 * 1e3 / args.steps,
                "roofline": {"bound": "alu", "achieved": ach32, "peak": PEAK_FP32_VALU_TFLOPS,
                             "unit": "TFLOP/s", "frac": ach32 / PEAK_FP32_VALU_TFLOPS,
                             "frac_of_unpacked_issue_rate": ach32 / PEAK_FP64_VALU_TFLOPS,
                             "kernel": "stage_kernel<float,16,16,true,false>", "avg_launch_us": stage32 * 1e6,
                             "note": "the published FP32 peak counts packed FP32 instructions, which this build "
                                     "does not emit; unpacked FP32 issues at the FP64 rate"},
                "l1_rel_density_err_vs_oracle": float(np.abs(U32[0].cpu().numpy() - final[0]).sum()
                                                      / np.abs(final[0]).sum()) if check else None,
                "err_steps": args.steps,
                "err_reference": "the FP64 state after the same steps, whose digest equals the oracle's"}
        log(f"fp32-bulk: {fp32['value']:.4e} cell-updates/s, {stage32 * 1e6:.2f} us per launch, "
            f"L1 rel density error {fp32['l1_rel_density_err_vs_oracle']}")
        s32.close()
    res = {"value": v64, "t64": t64, "runs": runs, "roofline": roof, "fp32": fp32,
           "fp64_digest_equals_oracle": check, "solver": s64, "prm": prm, "U0": U0, "grav": grav}
    return res


def cpu_leg(torch, hydro, head, steps_all, steps_one):
    """The oracle on the host: the headline workload's first steps on all the
    cores OpenMP is given and on one, each state compared bit for bit with the
    GPU's after as many steps."""
    import oracle
    prm, U0, grav = head["prm"], head["U0"], head["grav"]
    ncell = prm["nx"] * prm["ny"]
    o = oracle.Oracle(prm, gravity=grav)
    keep = oracle.threads()
    out = {}
    try:
        for key, nthreads, steps in (("all", keep, steps_all), ("one", 1, steps_one)):
            if steps <= 0:
                continue
            used = oracle.set_threads(nthreads)
            c0 = time.perf_counter()
            ref, _, _, _ = o.run(U0, steps)
            ct = time.perf_counter() - c0
            U = torch.tensor(U0, dtype=torch.float64, device="cuda")
            head["solver"].run(U, steps)
            out[key] = {"value": ncell * steps / ct, "threads": used, "steps": steps, "seconds": ct,
                        "fp64_bitwise_equal": bool(np.array_equal(U.cpu().numpy(), ref))}
            log(f"oracle ({used} threads): {out[key]['value']:.4e} cell-updates/s over {steps} steps "
                f"({ct:.1f} s), GPU bitwise {out[key]['fp64_bitwise_equal']}")
    finally:
        oracle.set_threads(keep)
    if "all" not in out:
        return None
    a = out["all"]
    cpu = {"value": a["value"], "unit": "cell-updates/s", "cores": a["threads"], "kind": "oracle",
           "sample": f"the first {a['steps']} SSP-RK3 steps of the same 1024^2 polytrope, C oracle with "
                     f"OpenMP over rows, columns and cells ({a['threads']} threads, {a['seconds']:.1f} s)",
           "fp64_bitwise_equal": a["fp64_bitwise_equal"], "host": host_cpu()}
    if "one" in out:
        o1 = out["one"]
        cpu["one_core"] = {"value": o1["value"], "cores": 1,
                           "sample": f"the first {o1['steps']} steps, one thread ({o1['seconds']:.1f} s)",
                           "fp64_bitwise_equal": o1["fp64_bitwise_equal"]}
    return cpu


def shear_layer_leg(torch, hydro, inputs, n, steps, warmup, cpu_steps, only_fp64):
    """The periodic shear layer (n^2, the 2000-step workload's grid): FP64 rate
    and stage roofline, FP32-bulk rate, and its error against the oracle after
    cpu_steps steps."""
    prm, U0 = inputs.kelvin_helmholtz(n, seed=2)
    ncell = n * n
    s64 = hydro.Solver(prm)
    U0d = torch.tensor(U0, dtype=torch.float64, device="cuda")
    U = U0d.clone()
    s64.run(U, warmup)
    U = U0d.clone()
    t64, _ = timed_run(torch, s64, U, steps)
    res = {"workload": f"kelvin_helmholtz_{n}x{n}", "steps": steps, "value": ncell * steps / t64,
           "ms_per_step": t64 * 1e3 / steps}
    res["roofline"] = stage_roofline(torch, s64, U0d, steps, ncell, FLOPS_PER_CELL_STAGE, BYTES_PER_CELL_STEP,
                                     f"kelvin_helmholtz_{n}x{n}", "stage_kernel<double,16,16,true,false>")
    log(f"shear layer {n}^2: {res['value']:.4e} cell-updates/s, {res['roofline']['avg_launch_us']:.2f} us per "
        f"launch ({res['roofline']['frac']:.3f} of the FP64 peak)")
    if not only_fp64:
        s32 = hydro.Solver(prm, precision=hydro.FP32_BULK)
        U32 = U0d.clone()
        s32.run(U32, warmup)
        U32 = U0d.clone()
        t32, _ = timed_run(torch, s32, U32, steps)
        res["fp32_value"] = ncell * steps / t32
        if cpu_steps > 0:
            import oracle
            ref, _, _, _ = oracle.Oracle(prm).run(U0, cpu_steps)
            U32 = U0d.clone()
            s32.run(U32, cpu_steps)
            res["fp32_l1_rel_density_err_vs_oracle"] = float(np.abs(U32[0].cpu().numpy() - ref[0]).sum()
                                                             / np.abs(ref[0]).sum())
            res["fp32_err_steps"] = cpu_steps
        s32.close()
    s64.close()
    return res


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


def adjoint_block(torch, hydro, inputs, args):
    """The adjoint workload in its stated form (FP32-bulk, checkpoints every
    ckpt steps: the headline ratio) and the other three forms; central
    differences of the FP64 gradient over every mode amplitude."""
    a_np = inputs.kh_sine_amplitudes()
    n, steps, ck = args.adj_n, args.adj_steps, args.adj_ckpt
    s64a, J64, g64, tf64, tb64, sched = adjoint_leg(torch, hydro, inputs, n, steps, None, hydro.FP64, a_np)
    _, J32, g32, tf32, tb32, _ = adjoint_leg(torch, hydro, inputs, n, steps, None, hydro.FP32_BULK, a_np, sched)
    _, _, g64c, tf64c, tb64c, _ = adjoint_leg(torch, hydro, inputs, n, steps, ck, hydro.FP64, a_np, sched)
    _, _, g32c, tf32c, tb32c, _ = adjoint_leg(torch, hydro, inputs, n, steps, ck, hydro.FP32_BULK, a_np, sched)
    comps = list(range(len(a_np))) if args.fd_all else [0, 17, 63]
    c0 = time.perf_counter()
    fd = fd_check(torch, inputs, s64a, a_np, sched, comps)
    fd_s = time.perf_counter() - c0
    rel = np.abs(fd - g64[comps]) / np.abs(g64[comps])
    adj = {"workload": f"kh_sine_{n}x{n}_{steps}steps",
           "ratio": tb32c / tf32c,
           "ratio_form": f"FP32-bulk, checkpoints every {ck} steps (backward incl. segment replay / forward)",
           "J": J64,
           "fwd_ms_fp32_ckpt": tf32c * 1e3, "bwd_ms_fp32_ckpt": tb32c * 1e3,
           "ratio_fp64_ckpt": tb64c / tf64c, "fwd_ms_fp64_ckpt": tf64c * 1e3, "bwd_ms_fp64_ckpt": tb64c * 1e3,
           "ratio_fp64_all_states": tb64 / tf64, "ratio_fp32_all_states": tb32 / tf32,
           "states_kept_gb": 3 * steps * 32 * n * n / 1e9, "ckpt_every": ck,
           "ckpt_grad_bitwise_equal_fp64": bool(np.array_equal(g64c, g64)),
           "ckpt_grad_bitwise_equal_fp32": bool(np.array_equal(g32c, g32)),
           "fd_components": len(comps), "fd_h": 1e-7, "fd_seconds": fd_s,
           "fd_rel_err_max": float(rel.max()), "fd_rel_err_median": float(np.median(rel)),
           "fd_rel_err_worst_component": int(comps[int(np.argmax(rel))]),
           "grad_rel_err_fp32_vs_fp64": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64)),
           "grad_rel_err_fp32_vs_fp64_max_component": float(np.max(np.abs(g32 - g64) / np.abs(g64)))}
    if args.cpu_steps > 0:
        # the plain-PyTorch reference adjoint (autograd through the textbook
        # step, FP64, on the host) of one step at full size from the initial
        # state, timed beside the GPU's and compared with it
        from oracle import torch_ref
        prm = inputs.kh_sine_params(n)
        U0 = np.ascontiguousarray(inputs.kh_sine_state(a_np, prm), dtype=np.float64)
        dt0, al0 = float(sched[0][0]), np.asarray(sched[1][0], dtype=np.float64)
        lam = np.random.default_rng(11).standard_normal(U0.shape)
        got = s64a.step_vjp(torch.tensor(U0, device="cuda"), dt0, al0,
                            torch.tensor(lam, device="cuda")).cpu().numpy()
        c0 = time.perf_counter()
        want = torch_ref.vjp(prm, None, U0, dt0, [tuple(r) for r in al0], lam)
        ct = time.perf_counter() - c0
        adj["cpu_reference"] = {
            "cell_step_vjps_per_s": n * n / ct, "cores": torch.get_num_threads(),
            "kind": "plain PyTorch autograd, FP64",
            "sample": f"one step's adjoint at full size from the initial state, {ct:.1f} s",
            "rel_err_l2_gpu_vs_reference": float(np.linalg.norm(got - want) / np.linalg.norm(want))}
        log(f"adjoint: reference step adjoint on the host {ct:.1f} s "
            f"({adj['cpu_reference']['cores']} threads), GPU relative error "
            f"{adj['cpu_reference']['rel_err_l2_gpu_vs_reference']:.1e}")
    log(f"adjoint: FP32 checkpointed ratio {adj['ratio']:.2f} (fwd {tf32c * 1e3:.1f} ms, bwd {tb32c * 1e3:.1f} ms); "
        f"FP64 checkpointed {adj['ratio_fp64_ckpt']:.2f}; all states {adj['ratio_fp64_all_states']:.2f} / "
        f"{adj['ratio_fp32_all_states']:.2f}; FD over {len(comps)} amplitudes: max rel err "
        f"{adj['fd_rel_err_max']:.2e} ({fd_s:.1f} s); fp32 grad rel err {adj['grad_rel_err_fp32_vs_fp64']:.2e}")
    return adj


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
    """The shear layer (2000 steps) and the heavy-over-light layer (5000 steps)
    at full length, FP64 and FP32-bulk: rates, the FP64 final state's digest
    against the oracle's, and the FP32 form's relative L1 density error against
    that state (the oracle's when the digests agree)."""
    cases = [("shear_layer_512", "kelvin_helmholtz_512x512_2000steps",
              lambda: inputs.kelvin_helmholtz(512, seed=2), 2000),
             ("heavy_over_light_256x1024", "rayleigh_taylor_256x1024_5000steps",
              lambda: inputs.rayleigh_taylor(), 5000)]
    out = []
    for key, name, make, steps in cases:
        prm, U0 = make()
        res = {"workload": name}
        fin = {}
        for prec, k in ((hydro.FP64, "fp64"), (hydro.FP32_BULK, "fp32")):
            s = hydro.Solver(prm, precision=prec)
            U = torch.tensor(U0, dtype=torch.float64, device="cuda")
            t, _ = timed_run(torch, s, U, steps)
            res[f"{k}_cell_updates_per_s"] = prm["nx"] * prm["ny"] * steps / t
            fin[k] = U.cpu().numpy()
            s.close()
        want = golden_state_digest(key, steps)
        res["fp64_digest_equals_oracle"] = None if want is None else bool(digest(fin["fp64"]) == want)
        d = np.abs(fin["fp32"][0] - fin["fp64"][0]).sum() / np.abs(fin["fp64"][0]).sum()
        res["fp32_l1_rel_density_err_vs_oracle" if res["fp64_digest_equals_oracle"]
            else "fp32_l1_rel_density_err_vs_fp64"] = float(d)
        log(f"config {name}: fp64 {res['fp64_cell_updates_per_s']:.3e}, fp32 {res['fp32_cell_updates_per_s']:.3e} "
            f"cell-updates/s, oracle digest {res['fp64_digest_equals_oracle']}, fp32 L1 err {d:.2e}")
        out.append(res)
    return out


def poisson_leg(torch, hydro, inputs, n, cpu_iters):
    """Potential of the n = 3 polytrope's density from a zero start to the
    relative change 1e-8 with the near-optimal over-relaxation factor."""
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
    us_it = t * 1e6 / iters
    out = {"workload": f"polytrope_density_{n}x{n}_zero_start_tol1e-8", "omega": omega,
           "iterations": iters, "last_change": change, "ms": t * 1e3, "wall_ms": wall * 1e3,
           "cell_iterations_per_s": n * n * iters / t, "us_per_iteration": us_it,
           "hbm_gbs_single_sweep_count": POISSON_BYTES_PER_CELL_ITER * n * n * iters / t / 1e9}
    pc = POISSON_COUNTERS
    if n == 1024 and sources_digest(pc["sources"]) == pc["sha256"]:
        k = pc["iterations_per_launch"]
        out["measured"] = {
            "hbm_bytes_per_cell_iteration": pc["bytes_per_launch"] / k / (n * n),
            "hbm_gbs_during_launch": pc["bytes_per_launch"] / (pc["launch_us"] * 1e-6) / 1e9,
            "issue_frac": pc["valu_insts_per_launch"] / (pc["launch_us"] * 1e-6) / PEAK_VALU_WAVE_INSTS_PER_S,
            "bound": "issue and LDS latency (temporal blocking keeps HBM traffic low)",
            "counters_launch_us": pc["launch_us"]}
    log(f"poisson: {iters} iterations in {t * 1e3:.1f} ms ({us_it:.2f} us/iteration)")
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
    for _ in range(steps):
        ev[0].record(st)
        s.ls_step(S, vel, s_f, dt)
        ev[1].record(st)
        s.ls_redistance(S, count=False)
        ev[2].record(st)
        torch.cuda.synchronize()
        t_step += ev[0].elapsed_time(ev[1]) / 1e3
        t_red += ev[1].elapsed_time(ev[2]) / 1e3
    npts = int(s.ls_front(S).shape[0])  # (of the field the last re-distancing left)
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
        # one re-distancing of the current field on both sides: the oracle's
        # brute force timed, the distances compared bit for bit
        S_host = S.cpu().numpy()
        dist = torch.zeros_like(S)
        s.ls_redistance(S, dist)
        c0 = time.perf_counter()
        _, want_d, want_n = ls.redistance(S_host)
        ct = time.perf_counter() - c0
        out["cpu_oracle_redistance"] = {
            "corners_per_s": nc / ct, "cores": 1, "front_points": want_n,
            "sample": f"one re-distancing at full size (brute force), {ct:.2f} s",
            "distances_bitwise_equal": bool(np.array_equal(dist.cpu().numpy(), want_d))}
        log(f"levelset: oracle re-distancing {ct:.2f} s (GPU {out['redistance_us']:.1f} us), "
            f"distances bitwise {out['cpu_oracle_redistance']['distances_bitwise_equal']}")
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000,
                    help="timed steps of the polytrope (its full length: 1000)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of K steps from the initial state (the first is the value)")
    ap.add_argument("--cpu-steps", type=int, default=40,
                    help="oracle steps of the polytrope timed on all cores (0: skip every CPU leg)")
    ap.add_argument("--cpu-steps-one", type=int, default=10, help="oracle steps timed on one thread")
    ap.add_argument("--only-fp64", action="store_true", help="skip the FP32-bulk legs")
    ap.add_argument("--only-headline", action="store_true", help="the polytrope only (for profiling)")
    ap.add_argument("--with-shear", action="store_true",
                    help="with --only-headline: also the shear-layer leg (FP64)")
    ap.add_argument("--kh-n", type=int, default=512, help="shear-layer leg grid (n x n; 0: skip)")
    ap.add_argument("--kh-steps", type=int, default=2000)
    ap.add_argument("--kh-cpu-steps", type=int, default=100,
                    help="oracle steps for the shear layer's FP32 error")
    ap.add_argument("--char-steps", type=int, default=400,
                    help="steps of the characteristic-reconstruction leg (0: skip)")
    ap.add_argument("--char-cpu-steps", type=int, default=3,
                    help="oracle steps of that leg compared bit for bit")
    ap.add_argument("--adj-n", type=int, default=1024, help="adjoint workload grid (n x n; 0: skip)")
    ap.add_argument("--adj-steps", type=int, default=500)
    ap.add_argument("--adj-ckpt", type=int, default=50, help="checkpoint interval of the adjoint")
    ap.add_argument("--fd-all", type=int, default=1,
                    help="central differences over all 64 amplitudes (0: three of them)")
    ap.add_argument("--poisson-n", type=int, default=1024,
                    help="potential-solver workload grid (n x n; 0: skip)")
    ap.add_argument("--poisson-cpu-iters", type=int, default=200)
    ap.add_argument("--ls-n", type=int, default=1024, help="level-set workload cells per side (0: skip)")
    ap.add_argument("--ls-steps", type=int, default=20)
    ap.add_argument("--sweep", type=str, default="2048,4096",
                    help="grid sizes of the out-of-cache sweep (comma separated; empty: skip)")
    ap.add_argument("--sweep-steps", type=int, default=200)
    ap.add_argument("--no-probes", action="store_true", help="skip the fma-rate and copy probes")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the full-length runs of the shear layer (2000 steps) and the "
                         "heavy-over-light layer (5000)")
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
    if args.only_headline:
        if not args.with_shear:
            args.kh_n = 0
        args.char_steps = args.adj_n = args.poisson_n = args.ls_n = 0
        args.sweep = ""
        args.no_probes = args.no_configs = True
        args.cpu_steps = 0

    head = headline_leg(torch, hydro, inputs, args)
    cpu = None
    if args.cpu_steps > 0:
        cpu = cpu_leg(torch, hydro, head, args.cpu_steps, args.cpu_steps_one)
    head["solver"].close()

    kh = None
    if args.kh_n > 0:
        kh = shear_layer_leg(torch, hydro, inputs, args.kh_n, args.kh_steps, 200,
                             args.kh_cpu_steps if args.cpu_steps > 0 else 0, args.only_fp64)
    adj = None if args.adj_n <= 0 else adjoint_block(torch, hydro, inputs, args)
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
        chw = charwise_leg(torch, hydro, inputs, 512, args.char_steps,
                           args.char_cpu_steps if args.cpu_steps > 0 else 0)
    lset = None
    if args.ls_n > 0:
        lset = levelset_leg(torch, hydro, inputs, args.ls_n, args.ls_steps, args.cpu_steps > 0)

    runs = head["runs"]
    out = {
        "metric": "cell-updates/sec per RK3 step FP64 vs FP32 at stated L1 err; adjoint/fwd ratio",
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["t64"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "polytrope_1024x1024_rz_1000steps", "nx": 1024, "ny": 1024,
                   "geometry": "cylindrical (r, z)", "gamma": 4.0 / 3.0, "cfl": 0.5,
                   "bc": "reflecting axis and plane, transmissive outside", "gravity": "fixed field",
                   "rho_floor": 1e-8, "seed": 4, "precision": "fp64",
                   "steps_from_initial_state": args.steps},
        "fp64_digest_equals_oracle": head["fp64_digest_equals_oracle"],
        "roofline": head["roofline"],
        "repeats": {"runs": len(runs), "median": float(np.median(runs)), "min": min(runs), "max": max(runs)},
        "cpu_baseline": cpu,
        "fp32_bulk": head["fp32"],
        "adjoint": adj,
        "shear_layer": kh,
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
