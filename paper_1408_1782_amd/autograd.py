"""Differentiable time integration: a torch.autograd.Function around the
library's splitting step (forward) and its adjoint step (reverse).

Forward: ``nsteps`` steps of qb_step, keeping a copy of the state every
``checkpoint_every`` steps.  Backward: for each segment, last to first, the
steps are run again from the segment's checkpoint with qb_step_trace (one
record per step: input state, Heun stage, Heun output), then qb_adjoint_step
walks the records backwards, carrying the state cotangent and accumulating
the cotangent of the field B.  Gradients follow torch's convention for
complex tensors (G = dl/dRe W + i dl/dIm W); all arithmetic runs in the HIP
library.
"""
import torch


class _Evolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W0, B, plan, dt, nsteps, every):
        W = W0.detach().clone().contiguous()
        Bd = None if B is None else B.detach().contiguous()
        ckpts = []
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            ckpts.append(W.clone())
            plan.step(W, Bd, dt, k)
            done += k
        ctx.plan, ctx.dt, ctx.nsteps, ctx.every = plan, dt, nsteps, every
        ctx.ckpts, ctx.B = ckpts, Bd
        return W

    @staticmethod
    def backward(ctx, gW):
        plan, dt, every = ctx.plan, ctx.dt, ctx.every
        lam = gW.detach().to(plan.cdtype).contiguous().clone()
        gB = torch.zeros((plan.problem.Nx, 3), dtype=torch.float64, device=lam.device)
        rb = plan.trace_bytes
        trace = plan.new_trace(min(every, ctx.nsteps))
        for s in reversed(range(len(ctx.ckpts))):
            k = min(every, ctx.nsteps - s * every)
            W = ctx.ckpts[s].clone()
            plan.step_trace(W, ctx.B, dt, k, trace)
            for n in reversed(range(k)):
                plan.adjoint_step(lam, ctx.B, dt, record=trace[n * rb:(n + 1) * rb], lam=lam, gB=gB)
        gB_out = gB if ctx.needs_input_grad[1] else None
        return lam, gB_out, None, None, None, None


def evolve(plan, W0, B, dt, nsteps, checkpoint_every=20):
    """W(T) after ``nsteps`` splitting steps of length dt from W0 in field B
    (float64 [Nx, 3] or None), differentiable in W0 and B."""
    if plan.trace_bytes == 0:
        raise ValueError("plan has no trace")
    plan.enable_adjoint()
    return _Evolve.apply(W0, B, plan, float(dt), int(nsteps), max(1, int(checkpoint_every)))
