"""Differentiable PIC runs: a torch.autograd.Function over the C ABI.

Forward: nsteps steps of a Sim (FP32 path, periodic grid) from initial fields
E0, B0 and initial momenta U0 (one (3, capacity) tensor per species, in the
storage order at the call), saving the full state every K steps.  With
sort=True the particles are also sorted (recording the permutation) at every
checkpoint, which is the counting sort every K steps of a long run; the
Sim's own periodic sort must then be off (sort_every=0).
Backward: for each checkpoint segment, from the last: re-compute the
segment's states from its checkpoint, each step written straight into the
next state's arrays (empic_step_state), apply the step adjoint
(empic_step_vjp) backwards through them, then the adjoint of the segment's
sort.  Memory: one saved state (and permutation) per K steps plus K - 1
states of the segment being reversed.  The Sim's fields hold a re-computed
state afterwards, not the final one.
"""
from __future__ import annotations

import torch


class PicRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, nsteps, K, sort, E0, B0, *U0):
        if sim.fp64:
            raise ValueError("differentiable runs use the FP32 path")
        if sim.sort_every != 0:
            raise ValueError("create the Sim with sort_every=0: a differentiable run sorts "
                             "at its checkpoints (sort=True)")
        if K < 1:
            raise ValueError("checkpoint interval K must be >= 1")
        with torch.no_grad():
            sim.E.copy_(E0)
            sim.B.copy_(B0)
            for i, u in enumerate(U0):
                sim.current_buffers(i)["u"].copy_(u)
            ckpts, perms = [], []
            for n in range(int(nsteps)):
                if n % K == 0:
                    perm = None
                    if sort:
                        perm = sim.alloc_perm()
                        sim.sort_recorded(perm)
                    perms.append(perm)
                    ckpts.append(sim.save_state())
                sim.step(1)
        ctx.sim, ctx.nsteps, ctx.K = sim, int(nsteps), int(K)
        ctx.ckpts, ctx.perms = ckpts, perms
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
            # slot 0 of a segment is its checkpoint; the re-computed states share
            # its ids and weights, which no step changes
            pool = [None] + [sim.alloc_state(particle_record=False)
                             for _ in range(min(K, nsteps) - 1)]
            for seg in reversed(range(len(ctx.ckpts))):
                start = seg * K
                stop = min(start + K, nsteps)
                ck = ctx.ckpts[seg]
                states = [ck]
                for j in range(1, stop - start):
                    st = dict(pool[j], id=ck["id"], w=ck["w"])
                    sim.step_state(states[-1], st)
                    states.append(st)
                for st in reversed(states):
                    sim.step_vjp(st, lam)
                if ctx.perms[seg] is not None:
                    sim.sort_vjp(ctx.perms[seg], lam)
        ctx.ckpts = ctx.perms = None
        return (None, None, None, None, lam["E"], lam["B"], *lam["u"])


def run(sim, nsteps, K, E0, B0, U0, sort=False):
    """Differentiable (E_N, B_{N-1/2}) of `nsteps` steps from (E0, B0, U0)."""
    return PicRun.apply(sim, nsteps, K, bool(sort), E0, B0, *U0)
