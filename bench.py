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
adjoint workload (sine-mode shear layer, 1024^2, 500 steps, checkpoints every
50: backward/forward time ratio in FP64 and FP32, central-difference check,
FP32-vs-FP64 gradient error).
"""
from __future__ import annotations

import argparse
import json
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
    respect to its mode amplitudes, by the hand-written adjoint (checkpointed
    rollout).  Returns (J, grad, forward seconds, backward seconds, schedule)."""
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

    once(min(steps, 2 * ckpt))  # warm-up (allocations, code objects)
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="grid size (n x n)")
    ap.add_argument("--cpu-steps", type=int, default=40,
                    help="oracle steps timed for the CPU baseline (0: skip)")
    ap.add_argument("--only-fp64", action="store_true", help="skip the FP32-bulk leg")
    ap.add_argument("--adj-n", type=int, default=1024, help="adjoint workload grid (n x n; 0: skip)")
    ap.add_argument("--adj-steps", type=int, default=500)
    ap.add_argument("--adj-ckpt", type=int, default=50)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB three times (a known-size "
                         "kernel for calibrating the profiler's HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
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

    # stage-kernel average duration: 3 stage launches per step (plus three tiny
    # set-up kernels per call, included, so the estimate is conservative)
    stage_s = t64 / (3 * args.steps)
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
        s64a, J64, g64, tf64, tb64, sched = adjoint_leg(torch, hydro, inputs, args.adj_n, args.adj_steps,
                                                       args.adj_ckpt, hydro.FP64, a_np)
        _, J32, g32, tf32, tb32, _ = adjoint_leg(torch, hydro, inputs, args.adj_n, args.adj_steps,
                                                 args.adj_ckpt, hydro.FP32_BULK, a_np, sched)
        comps = [0, 17, 63]
        fd = fd_check(torch, inputs, s64a, a_np, sched, comps)
        fd_err = float(np.max(np.abs(fd - g64[comps]) / np.abs(g64).max()))
        adj = {"workload": f"kh_sine_{args.adj_n}x{args.adj_n}_{args.adj_steps}steps_ckpt{args.adj_ckpt}",
               "J": J64,
               "fwd_ms_fp64": tf64 * 1e3, "bwd_ms_fp64": tb64 * 1e3, "ratio_fp64": tb64 / tf64,
               "fwd_ms_fp32": tf32 * 1e3, "bwd_ms_fp32": tb32 * 1e3, "ratio_fp32": tb32 / tf32,
               "fd_components": comps, "fd_rel_err_fp64": fd_err,
               "grad_rel_err_fp32_vs_fp64": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))}
        log(f"adjoint: fp64 ratio {adj['ratio_fp64']:.2f} (fwd {tf64 * 1e3:.1f} ms, bwd {tb64 * 1e3:.1f} ms), "
            f"fp32 ratio {adj['ratio_fp32']:.2f}, FD rel err {fd_err:.2e}, "
            f"fp32 grad rel err {adj['grad_rel_err_fp32_vs_fp64']:.2e}")

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
                     "traffic": None, "kernel": "stage_kernel<double,16,16>",
                     "avg_launch_us": stage_s * 1e6, "hbm_gbs_algorithmic": hbm_gbs,
                     "hbm_frac": hbm_gbs / PEAK_HBM_GBS},
        "cpu_baseline": cpu,
        "fp32_bulk": fp32,
        "adjoint": adj,
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
