"""Differentiable multi-step rollout: forward with dg_run, backward with the
discrete adjoint of each step (dg_adjoint_step) and checkpointed recomputation.

Forward: n SSP-RK2 steps from U0 (adaptive CFL step sizes, or a given
schedule), storing the state every k steps (the stage-2 kernel writes the
checkpoint directly; no copy).  The step sizes are part of the output and are
treated as constants by the backward pass (dt frozen: the gradient is that of
the discrete map with the recorded schedule).

Backward, segment by segment from the last: recompute the segment's states
U^s .. U^(e-1) and stage-1 outputs V1^s .. V1^(e-1) from its checkpoint (one
dg_run with every state kept, plus one stage 1), then apply
lam^n = (dS/dU^n)^T lam^(n+1) for n = e-1 .. s.  Memory: the checkpoints
plus 2k states for one segment.
"""
from __future__ import annotations

import torch

from .solver import Solver


class DGRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0: torch.Tensor, solver: Solver, nsteps: int, cfl: float, k: int,
                dt_hist: torch.Tensor | None, graph: bool):
        if k < 1:
            raise ValueError("checkpoint interval k must be >= 1")
        U0 = U0.detach()
        nck = (nsteps - 1) // k
        ckpts = [solver.empty() for _ in range(nck)]
        if dt_hist is None:
            out, dt_hist = solver.run(U0, nsteps, cfl=cfl, ckpt_every=k, ckpts=ckpts, graph=graph)
        else:
            out, dt_hist = solver.run(U0, nsteps, cfl=0.0, dt_hist=dt_hist.detach(), ckpt_every=k,
                                      ckpts=ckpts, graph=graph)
        ctx.solver, ctx.nsteps, ctx.k, ctx.graph = solver, nsteps, k, graph
        ctx.save_for_backward(U0, dt_hist, *ckpts)
        ctx.mark_non_differentiable(dt_hist)
        return out, dt_hist

    @staticmethod
    def backward(ctx, lam_out, _unused):
        solver, nsteps, k = ctx.solver, ctx.nsteps, ctx.k
        U0, dt_hist, *ckpts = ctx.saved_tensors
        ni = solver.ninst
        lam = lam_out.to(solver.dtype).contiguous()
        lam_b = solver.empty()
        Useg = [solver.empty() for _ in range(max(k - 1, 0))]
        V1 = [solver.empty() for _ in range(k)]
        nseg = (nsteps + k - 1) // k

        def dt(n):
            return dt_hist[n * ni:(n + 1) * ni]

        for j in range(nseg - 1, -1, -1):
            s, e = j * k, min((j + 1) * k, nsteps)
            m = e - s
            start = U0 if j == 0 else ckpts[j - 1]
            states = [start] + Useg[:m - 1]
            if m >= 2:
                solver.run(start, m - 1, cfl=0.0, dt_hist=dt_hist[s * ni:(e - 1) * ni],
                           out=Useg[m - 2], ckpt_every=1, ckpts=Useg[:m - 2],
                           v1_keep=V1[:m - 1], graph=ctx.graph)
            solver.stage1(states[m - 1], dt(e - 1), V1[m - 1])
            for n in range(e - 1, s - 1, -1):
                solver.adjoint_step(states[n - s], dt(n), lam, V1=V1[n - s], out=lam_b)
                lam, lam_b = lam_b, lam
        return lam, None, None, None, None, None, None


def rollout(solver: Solver, U0: torch.Tensor, nsteps: int, cfl: float = 0.3, k: int = 20,
            dt_hist: torch.Tensor | None = None, graph: bool = True):
    """(U_n, dt_hist) after nsteps steps; differentiable in U0 (dt frozen).
    With dt_hist given ((nsteps) x ninst step sizes) the schedule is fixed."""
    return DGRollout.apply(U0, solver, int(nsteps), float(cfl), int(k), dt_hist, bool(graph))
