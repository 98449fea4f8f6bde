"""Differentiable PIC runs: a torch.autograd.Function over the C ABI.

Forward: nsteps steps of a Sim (FP32 path, periodic grid, no sort inside the
run) from initial fields E0, B0 and initial momenta U0 (one (3, capacity)
tensor per species, storage order), saving the full state every K steps.
Backward: for each checkpoint segment, from the last: reload its state,
recompute the segment's states, then apply the step adjoint
(empic_step_vjp) backwards through them.  Memory: one saved state per K
steps plus K states of the segment being reversed.
"""
from __future__ import annotations

import torch


class PicRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, nsteps, K, E0, B0, *U0):
        if sim.fp64:
            raise ValueError("differentiable runs use the FP32 path")
        with torch.no_grad():
            sim.E.copy_(E0)
            sim.B.copy_(B0)
            for i, u in enumerate(U0):
                sim.current_buffers(i)["u"].copy_(u)
            ckpts = []
            for n in range(int(nsteps)):
                if n % K == 0:
                    ckpts.append(sim.save_state())
                sim.step(1)
        ctx.sim, ctx.nsteps, ctx.K, ctx.ckpts = sim, int(nsteps), int(K), ckpts
        return sim.E.clone(), sim.B.clone()

    @staticmethod
    def backward(ctx, gE, gB):
        sim, nsteps, K = ctx.sim, ctx.nsteps, ctx.K
        lam = sim.alloc_adjoint()
        with torch.no_grad():
            if gE is not None:
                lam["E"].copy_(gE)
            if gB is not None:
                lam["B"].copy_(gB)
            pool = [sim.alloc_state() for _ in range(K)]
            for seg in reversed(range(len(ctx.ckpts))):
                start = seg * K
                stop = min(start + K, nsteps)
                sim.load_state(ctx.ckpts[seg])
                states = [ctx.ckpts[seg]]
                for j in range(1, stop - start):
                    sim.step(1)
                    states.append(sim.save_state(pool[j]))
                for st in reversed(states):
                    sim.step_vjp(st, lam)
        ctx.ckpts = None
        return (None, None, None, lam["E"], lam["B"], *lam["u"])


def run(sim, nsteps, K, E0, B0, U0):
    """Differentiable (E_N, B_{N-1/2}) of `nsteps` steps from (E0, B0, U0)."""
    return PicRun.apply(sim, nsteps, K, E0, B0, *U0)
