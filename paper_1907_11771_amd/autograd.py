"""Differentiable receiver traces of a run of extrapolated GBS macro steps.

    traces = receiver_traces(plan, y0, c2, n_macro, t0=0.0, checkpoint_every=20,
                             keep_pairs=None)

``traces[m, r]`` is the pressure at receiver r after macro step m+1.  The
backward pass is the library's hand-written adjoint (gbs_adjoint_step): the
forward pass keeps the state at every ``checkpoint_every``-th macro-step
boundary, and the backward pass recomputes the states of one segment at a
time from its checkpoint, then runs the adjoint macro steps of the segment
in reverse, injecting the traces' gradients.  Gradients: the initial state
y0 and the coefficient field c^2 (accumulated in FP64).

With the temporally blocked adjoint (2-D FD4), the recomputation of a
segment can also keep the last two leap-frog levels of every sequence and
macro step (gbs_step_keep_pairs), so that the adjoint steps do not rebuild
them (gbs_adjoint_step_pairs): 2 k states per macro step of the segment.
keep_pairs=None does this when that buffer takes at most a quarter of the
free device memory, True always, False never.  The adjoint steps from kept
levels run on ``plan.adjoint_lanes`` streams when set (autotune_adjoint).

The plan's coefficient field is shared by all calls on the plan: each
forward copies its c^2 into it and keeps a copy, and each backward puts that
copy back first, so forwards of other c^2 between a forward and its backward
(a line search, a sum of losses) do not change the gradient.  After a
backward the field holds that backward's c^2.
"""
import torch

from .plan import GBSPlan


class _ReceiverTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, c2, plan, n_macro, t0, checkpoint_every, keep_pairs):
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
        ctx.keep_pairs = keep_pairs
        ctx.cps = cps
        # the plan's field is shared by every call on the plan: keep this
        # forward's c^2, which the backward pass puts back before recomputing
        ctx.c2_fwd = plan.c2_field.clone()
        ctx.y0_dtype, ctx.c2_dtype = y0.dtype, c2.dtype
        return traces[:, :getattr(plan, "n_rec", 0)].to(y0.dtype)

    @staticmethod
    def backward(ctx, gtr):
        plan, n, t0, ck = ctx.plan, ctx.n_macro, ctx.t0, ctx.ck
        plan.c2_field.copy_(ctx.c2_fwd)
        gtr = gtr.to(plan.dtype).contiguous()
        ybar = torch.zeros_like(ctx.cps[0])
        grad = torch.zeros(plan.c2_field.shape, dtype=torch.float64, device=plan.device)
        starts = list(range(0, n, ck))
        pairs = _pairs_buffer(plan, min(ck, n), ctx.keep_pairs)
        for s in reversed(starts):
            e = min(s + ck, n)
            # states at the start of macro steps s .. e-1 (and, kept, the last
            # two levels of every sequence of each of those macro steps)
            states = [ctx.cps[s]]
            y = ctx.cps[s].clone()
            for m in range(s, e):
                if pairs is not None:
                    plan.step_keep_pairs(y, y, pairs[m - s:m - s + 1], t0=t0 + m * plan.H)
                elif m < e - 1:
                    plan.step(y, y, t0=t0 + m * plan.H, n_macro=1)
                if m < e - 1:
                    states.append(y.clone())
            fwd_lanes = plan.lanes
            if pairs is not None and plan.adjoint_lanes:
                plan.set_lanes(plan.adjoint_lanes)
            try:
                for m in range(e - 1, s - 1, -1):
                    if pairs is not None:
                        plan.adjoint_step_pairs(t0 + m * plan.H, states[m - s], pairs[m - s],
                                                ybar, trace_bar=gtr[m], grad_c2=grad)
                    else:
                        plan.adjoint_step(t0 + m * plan.H, states[m - s], ybar,
                                          trace_bar=gtr[m], grad_c2=grad)
            finally:
                # the forward's stream count, also when an adjoint step raises
                plan.set_lanes(fwd_lanes)
        ctx.cps = None
        ctx.c2_fwd = None
        return ybar.to(ctx.y0_dtype), grad.to(ctx.c2_dtype), None, None, None, None, None


def _pairs_buffer(plan, seg, keep):
    """The kept-levels buffer for a segment of ``seg`` macro steps, or None."""
    if keep is False or not plan.blocked_adjoint():
        return None
    shape = plan.pairs_shape(seg)
    nbytes = torch.Size(shape).numel() * torch.empty((), dtype=plan.dtype).element_size()
    if keep is None:
        free, _ = torch.cuda.mem_get_info(plan.device)
        if nbytes > free // 4:
            return None
    return torch.empty(shape, dtype=plan.dtype, device=plan.device)


def receiver_traces(plan: GBSPlan, y0, c2, n_macro, t0=0.0, checkpoint_every=20,
                    keep_pairs=None):
    return _ReceiverTraces.apply(y0, c2, plan, int(n_macro), float(t0), int(checkpoint_every),
                                 keep_pairs)
