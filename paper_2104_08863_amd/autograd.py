"""Differentiable projection steps on top of the hand-written adjoint.

ProjectionStep: one step as a torch.autograd.Function; the backward pass calls
the library's adjoint (transposed momentum stencils and the pressure solve
applied to g / W, using the self-adjointness of the discrete Poisson operator in
the face-volume inner product) -- nothing is traced by autograd.

rollout(): n steps with checkpoints every k steps; the backward pass
recomputes each k-step segment from its checkpoint and runs the step adjoints
in reverse.  The forward kernels are deterministic, so the recomputed states
and therefore the gradient are bitwise the same as without checkpointing.
"""
from __future__ import annotations

import torch


class ProjectionStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, dt, nu, fx, u, v, w):
        u, v, w = (t.contiguous() for t in (u, v, w))
        out = plan.projection_step(u, v, w, dt, nu, fx)
        ctx.plan, ctx.params = plan, (dt, nu, fx)
        ctx.save_for_backward(u, v, w)
        return out

    @staticmethod
    def backward(ctx, gu1, gv1, gw1):
        u, v, w = ctx.saved_tensors
        plan = ctx.plan
        g1 = tuple(torch.zeros_like(u) if g is None else g.contiguous() for g in (gu1, gv1, gw1))
        g = plan.projection_step_adjoint(u, v, w, *g1, *ctx.params)
        return (None, None, None, None) + tuple(g)


def projection_step(plan, u, v, w, dt, nu, fx):
    return ProjectionStep.apply(plan, dt, nu, fx, u, v, w)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, nsteps, every, dt, nu, fx, u, v, w):
        state = tuple(t.contiguous() for t in (u, v, w))
        ckpts = []
        for n in range(nsteps):
            if n % every == 0:
                ckpts.append(tuple(t.clone() for t in state))
            state = plan.projection_step(*state, dt, nu, fx)
        ctx.plan, ctx.nsteps, ctx.every, ctx.params = plan, nsteps, every, (dt, nu, fx)
        ctx.save_for_backward(*[t for c in ckpts for t in c])
        return state

    @staticmethod
    def backward(ctx, gu, gv, gw):
        plan, nsteps, every, params = ctx.plan, ctx.nsteps, ctx.every, ctx.params
        flat = ctx.saved_tensors
        ckpts = [flat[3 * i:3 * i + 3] for i in range(len(flat) // 3)]
        g = tuple(torch.zeros_like(flat[0]) if x is None else x.contiguous() for x in (gu, gv, gw))
        for seg in reversed(range(len(ckpts))):
            start = seg * every
            end = min(nsteps, start + every)
            states = [ckpts[seg]]
            for _ in range(start, end - 1):
                states.append(plan.projection_step(*states[-1], *params))
            for n in reversed(range(start, end)):
                g = plan.projection_step_adjoint(*states[n - start], *g, *params)
        return (None,) * 6 + tuple(g)


def rollout(plan, u, v, w, nsteps: int, dt: float, nu: float, fx: float, checkpoint_every: int = 1):
    """nsteps projection steps; differentiable w.r.t. (u, v, w) with step
    checkpointing every `checkpoint_every` steps."""
    if nsteps < 1 or checkpoint_every < 1:
        raise ValueError("nsteps and checkpoint_every must be >= 1")
    return _Rollout.apply(plan, int(nsteps), int(checkpoint_every), float(dt), float(nu), float(fx), u, v, w)
