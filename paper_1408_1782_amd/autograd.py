"""Differentiable time integration: a torch.autograd.Function around the
library's splitting step (forward) and its adjoint step (reverse).

Forward: ``nsteps`` steps of qb_step, keeping a copy of the state at the
start of every segment of ``checkpoint_every`` steps; the last segment runs
with qb_step_trace and keeps its step records (one per step: input state,
Heun stage, Heun output).  Backward: segments last to first; each earlier
segment is run again from its checkpoint with qb_step_trace, then
qb_adjoint_step walks the records backwards, carrying the state cotangent
and accumulating the cotangent of the field B.  ``checkpoint_every = 0``
keeps the records of every step instead (no recomputation; memory
nsteps * qb_trace_bytes).  Gradients follow torch's convention for complex
tensors (G = dl/dRe W + i dl/dIm W); all arithmetic runs in the HIP library.
"""
import torch


class _Evolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W0, B, plan, dt, nsteps, every):
        W = W0.detach().clone().contiguous()
        Bd = None if B is None else B.detach().contiguous()
        seg = nsteps if every <= 0 else every
        starts = list(range(0, nsteps, seg)) if nsteps > 0 else []
        ckpts = []
        last_trace = None
        for i, s0 in enumerate(starts):
            k = min(seg, nsteps - s0)
            ckpts.append(W.clone())
            if i == len(starts) - 1:
                last_trace = plan.new_trace(k)
                plan.step_trace(W, Bd, dt, k, last_trace)
            else:
                plan.step(W, Bd, dt, k)
        ctx.plan, ctx.dt, ctx.nsteps, ctx.seg = plan, dt, nsteps, seg
        ctx.starts, ctx.ckpts, ctx.B, ctx.last_trace = starts, ckpts, Bd, last_trace
        return W

    @staticmethod
    def backward(ctx, gW):
        plan, dt, seg = ctx.plan, ctx.dt, ctx.seg
        lam = gW.detach().to(plan.cdtype).contiguous().clone()
        gB = torch.zeros((plan.problem.Nx, 3), dtype=torch.float64, device=lam.device)
        rb = plan.trace_bytes
        trace = None
        for i in reversed(range(len(ctx.starts))):
            k = min(seg, ctx.nsteps - ctx.starts[i])
            if i == len(ctx.starts) - 1:
                rec = ctx.last_trace
            else:
                if trace is None:
                    trace = plan.new_trace(seg)
                W = ctx.ckpts[i].clone()
                plan.step_trace(W, ctx.B, dt, k, trace)
                rec = trace
            for n in reversed(range(k)):
                plan.adjoint_step(lam, ctx.B, dt, record=rec[n * rb:(n + 1) * rb], lam=lam, gB=gB)
        ctx.last_trace = None
        gB_out = gB if ctx.needs_input_grad[1] else None
        return lam, gB_out, None, None, None, None


def evolve(plan, W0, B, dt, nsteps, checkpoint_every=20):
    """W(T) after ``nsteps`` splitting steps of length dt from W0 in field B
    (float64 [Nx, 3] or None), differentiable in W0 and B.  Checkpoints every
    ``checkpoint_every`` steps (0: keep every step's record instead)."""
    plan.enable_adjoint()
    return _Evolve.apply(W0, B, plan, float(dt), int(nsteps), int(checkpoint_every))
