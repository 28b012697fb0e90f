"""Differentiable receiver traces of a run of extrapolated GBS macro steps.

    traces = receiver_traces(plan, y0, c2, n_macro, t0=0.0, checkpoint_every=20)

``traces[m, r]`` is the pressure at receiver r after macro step m+1.  The
backward pass is the library's hand-written adjoint (gbs_adjoint_step): the
forward pass keeps the state at every ``checkpoint_every``-th macro-step
boundary, and the backward pass recomputes the states of one segment at a
time from its checkpoint, then runs the adjoint macro steps of the segment
in reverse, injecting the traces' gradients.  Gradients: the initial state
y0 and the coefficient field c^2 (accumulated in FP64).
"""
import torch

from .plan import GBSPlan


class _ReceiverTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, c2, plan, n_macro, t0, checkpoint_every):
        if plan.c2_field is None:
            raise ValueError("the plan must have a coefficient field")
        plan.c2_field.copy_(c2.detach().to(plan.c2_field.dtype))
        y = y0.detach().to(plan.dtype).contiguous().clone()
        cps = {0: y.clone()}
        traces = torch.empty((n_macro, max(getattr(plan, "n_rec", 0), 1)), dtype=plan.dtype,
                             device=plan.device)
        # one library call per checkpoint segment
        for s in range(0, n_macro, checkpoint_every):
            e = min(s + checkpoint_every, n_macro)
            plan.step_record(y, y, t0=t0 + s * plan.H, n_macro=e - s, traces=traces[s:e])
            if e < n_macro:
                cps[e] = y.clone()
        ctx.plan, ctx.n_macro, ctx.t0, ctx.ck = plan, n_macro, t0, checkpoint_every
        ctx.cps = cps
        ctx.y0_dtype, ctx.c2_dtype = y0.dtype, c2.dtype
        return traces[:, :getattr(plan, "n_rec", 0)].to(y0.dtype)

    @staticmethod
    def backward(ctx, gtr):
        plan, n, t0, ck = ctx.plan, ctx.n_macro, ctx.t0, ctx.ck
        gtr = gtr.to(plan.dtype).contiguous()
        ybar = torch.zeros_like(ctx.cps[0])
        grad = torch.zeros(plan.c2_field.shape, dtype=torch.float64, device=plan.device)
        starts = list(range(0, n, ck))
        for s in reversed(starts):
            e = min(s + ck, n)
            # states at the start of macro steps s .. e-1
            states = [ctx.cps[s]]
            y = ctx.cps[s].clone()
            for m in range(s, e - 1):
                plan.step(y, y, t0=t0 + m * plan.H, n_macro=1)
                states.append(y.clone())
            for m in range(e - 1, s - 1, -1):
                plan.adjoint_step(t0 + m * plan.H, states[m - s], ybar, trace_bar=gtr[m],
                                  grad_c2=grad)
        ctx.cps = None
        return ybar.to(ctx.y0_dtype), grad.to(ctx.c2_dtype), None, None, None, None


def receiver_traces(plan: GBSPlan, y0, c2, n_macro, t0=0.0, checkpoint_every=20):
    return _ReceiverTraces.apply(y0, c2, plan, int(n_macro), float(t0), int(checkpoint_every))
