"""Differentiable rollouts over the HIP solver (torch.autograd).

:class:`HydroRollout` advances a state ``nsteps`` SSP-RK3 steps with the
device-side CFL step, recording each step's time step and the LF speeds of
its three stages, and keeps a checkpoint of the state every ``ckpt_every``
steps.  Its backward pass walks the segments from last to first: it re-runs
the segment from its checkpoint with the recorded schedule (bit-identical to
the forward) through ``hydro_step_save``, keeping the state at the start of
every step and its two Runge-Kutta stage states, and then applies
``hydro_step_vjp_saved`` step by step.  The last segment needs no re-run: the
forward pass runs it with ``hydro_run_save`` into the buffer the backward
pass replays into.  Memory: nsteps / ckpt_every checkpoints plus 3 *
ckpt_every states (that buffer, held from the forward pass to the end of the
backward pass).  With ``ckpt_every=None`` the forward
runs ``hydro_run_save`` and keeps all 3 * nsteps states (a 1024^2, 500-step
rollout: 50 GB, a sixth of the device's memory), and the backward pass is
the step adjoints alone.

The gradient is that of the discrete map with the schedule (dt and alpha of
every stage) held at its recorded values: those come from maxima over the
grid, and are treated as constants, as in any frozen-schedule adjoint.
"""
from __future__ import annotations

import torch

from . import hydro


class HydroRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver: "hydro.Solver", nsteps: int, ckpt_every=50):
        U = U0.detach().clone().contiguous()
        dts = torch.empty(max(nsteps, 1), dtype=torch.float64, device=U.device)
        als = torch.empty((max(nsteps, 1), 6), dtype=torch.float64, device=U.device)
        ctx.solver = solver
        ctx.nsteps = nsteps
        ctx.sched = (dts[:nsteps], als[:nsteps])
        if ckpt_every is None:
            # keep every step's start and stage states: no replay in backward
            states = torch.empty((max(nsteps, 1), 3) + tuple(U.shape), dtype=torch.float64, device=U.device)
            if nsteps > 0:
                solver.run_save(U, nsteps, states[:nsteps], dts[:nsteps], als[:nsteps])
            ctx.states = states
            ctx.ckpt_every = None
            return U
        if ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1 (or None to keep every state)")
        ckpts = []
        kmax = min(ckpt_every, nsteps)
        # the backward pass's replay buffer (each step's start state and two
        # stage states), filled here for the last segment, which the backward
        # pass then starts from without a replay
        pool = torch.empty((max(kmax, 1), 3) + tuple(U.shape), dtype=torch.float64, device=U.device)
        for s0 in range(0, nsteps, ckpt_every):
            k = min(ckpt_every, nsteps - s0)
            ckpts.append(U.clone())
            if s0 + k < nsteps:
                solver.run_into(U, k, dts[s0:s0 + k], als[s0:s0 + k])
            else:
                solver.run_save(U, k, pool[:k], dts[s0:s0 + k], als[s0:s0 + k])
        ctx.ckpt_every = ckpt_every
        ctx.ckpts = ckpts
        ctx.pool = pool
        ctx.pool_holds_last = True
        return U

    @staticmethod
    def backward(ctx, gU):
        solver = ctx.solver
        dts, als = ctx.sched
        dts_h = dts.cpu().numpy()
        als_h = als.cpu().numpy().reshape(-1, 2, 3).transpose(0, 2, 1)  # [n][stage][ax, ay]
        lam = gU.detach().contiguous().clone()
        nxt = torch.empty_like(lam)
        if ctx.ckpt_every is None:
            st = ctx.states
            for i in range(ctx.nsteps - 1, -1, -1):
                solver.step_vjp_saved(st[i, 0], st[i, 1], st[i, 2], dts_h[i], als_h[i], lam, out=nxt)
                lam, nxt = nxt, lam
            return lam, None, None, None
        # per step of a segment: its start state and its two stage states; the
        # forward pass left the last segment's there
        pool = ctx.pool
        nseg = len(ctx.ckpts)
        for seg in range(nseg - 1, -1, -1):
            s0 = seg * ctx.ckpt_every
            k = min(ctx.ckpt_every, ctx.nsteps - s0)
            if seg < nseg - 1 or not ctx.pool_holds_last:  # replay the segment from its checkpoint
                pool[0, 0].copy_(ctx.ckpts[seg])
                for i in range(k):
                    U, U1, U2 = pool[i, 0], pool[i, 1], pool[i, 2]
                    # the last step's end state is not needed, only its stages
                    dst = pool[i + 1, 0] if i + 1 < k else nxt
                    solver.step_save(U, dts_h[s0 + i], als_h[s0 + i], U1, U2, out=dst)
            for i in range(k - 1, -1, -1):
                U, U1, U2 = pool[i, 0], pool[i, 1], pool[i, 2]
                solver.step_vjp_saved(U, U1, U2, dts_h[s0 + i], als_h[s0 + i], lam, out=nxt)
                lam, nxt = nxt, lam
        ctx.pool_holds_last = False  # (a second backward pass replays every segment)
        return lam, None, None, None


def rollout(U0, solver, nsteps, ckpt_every=50):
    """Differentiable nsteps-step rollout of U0 (float64, (4, ny, nx), on the solver's device).
    ckpt_every=None keeps all 3 * nsteps states (96 B per cell and step) and the
    backward pass replays nothing."""
    return HydroRollout.apply(U0, solver, nsteps, ckpt_every)


class HydroStep(torch.autograd.Function):
    """One differentiable step with a given dt and (3, 2) LF speeds."""

    @staticmethod
    def forward(ctx, U, solver, dt, alpha):
        out = U.detach().clone().contiguous()
        solver.step(out, dt, alpha=alpha)
        ctx.save_for_backward(U.detach().contiguous())
        ctx.solver, ctx.dt, ctx.alpha = solver, dt, alpha
        return out

    @staticmethod
    def backward(ctx, g):
        (U,) = ctx.saved_tensors
        return ctx.solver.step_vjp(U, ctx.dt, ctx.alpha, g.contiguous()), None, None, None
