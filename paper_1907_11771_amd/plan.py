"""A torch-facing wrapper of one library plan: device memory (workspace,
coefficient field) comes from torch, kernels are enqueued on torch's current
HIP stream (a plan follows the current stream: every call that enqueues work
first rebinds the library plan when torch's current stream has changed,
gbs_plan_set_stream).  No arithmetic of the method happens here."""
import ctypes

import torch

from . import binding as B

_DT = {torch.float64: B.F64, torch.float32: B.F32}
_FIELDS = {B.ADVECT1D: 1, B.ACOUSTIC2D: 3, B.ACOUSTIC3D: 4}
_TEMPORAL = (B.VARIANT_TEMPORAL, B.VARIANT_TEMPORAL4, B.VARIANT_TEMPORAL_S5,
             B.VARIANT_TEMPORAL_S6, B.VARIANT_TEMPORAL_WG4, B.VARIANT_TEMPORAL_WG8)


def scheme_weights(scheme):
    """(steps, FP64 weights, ISB) of a scheme spec {p, steps, free_idx, c_free}
    with c_free given as "num/den" strings."""
    pairs = []
    for s in scheme["c_free"]:
        num, den = str(s).split("/")
        pairs.append((int(num), int(den)))
    w, isb = B.weights(scheme["p"], scheme["steps"], scheme["free_idx"], pairs)
    return list(scheme["steps"]), w, isb


class GBSPlan:
    """op: B.ADVECT1D / B.ACOUSTIC2D / B.ACOUSTIC3D; n: grid sizes (x[, y[, z]])."""

    def __init__(self, op, n, p, steps, w, H, fd_order=4, n_rhs=1, dtype=torch.float64,
                 c2=1.0, c2_field=None, c_max=None, device="cuda", check_stability=True):
        if not torch.cuda.is_available():
            raise RuntimeError("GBSPlan needs a HIP device; there is no CPU path")
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("GBSPlan runs on a HIP device, not %s" % self.device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dtype = dtype
        self.op, self.n, self.n_rhs = op, tuple(int(x) for x in n), n_rhs
        self.H = float(H)
        self.steps, self.w, self.p = list(steps), list(w), p
        flags = 0 if check_stability else B.FLAG_NO_STABILITY_CHECK
        self.c2_field = None
        ptr = None
        if c2_field is not None:
            self.c2_field = c2_field.to(device=self.device, dtype=dtype).contiguous()
            ptr = self.c2_field.data_ptr()
            if c_max is None:
                c_max = float(self.c2_field.max().sqrt())
        self.problem = B.make_problem(op, self.n, fd_order, n_rhs, _DT[dtype], c2, ptr,
                                      c_max or 0.0, flags)
        self.scheme = B.make_scheme(p, steps, w)
        nbytes = B.workspace_bytes(self.problem, self.scheme)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.handle = B.plan_create(self.problem, self.scheme, self.H, self.workspace.data_ptr(),
                                    self.workspace.numel(), self.stream.cuda_stream)
        self.lanes = 1               # streams of the forward passes
        self.adjoint_lanes = None    # streams of the adjoint passes (None: as the forward)

    @property
    def state_shape(self):
        return (self.n_rhs, _FIELDS[self.op]) + tuple(reversed(self.n))

    def _bind_stream(self):
        """Enqueue on torch's current stream of the plan's device."""
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            B.check(B.lib().gbs_plan_set_stream(self.handle, cur.cuda_stream))
            self.stream = cur

    def _check_state(self, t):
        if t.device != self.device or t.dtype != self.dtype or not t.is_contiguous():
            raise ValueError("state must be a contiguous %s tensor on %s" % (self.dtype, self.device))
        if t.numel() != int(torch.Size(self.state_shape).numel()):
            raise ValueError("state must have %s elements laid out as %s"
                             % (torch.Size(self.state_shape).numel(), self.state_shape))

    def step(self, y, out=None, t0=0.0, n_macro=1):
        """n_macro macro steps from time t0; returns the output tensor (``out``
        may be ``y`` itself)."""
        self._bind_stream()
        self._check_state(y)
        if out is None:
            out = torch.empty_like(y)
        self._check_state(out)
        B.check(B.lib().gbs_step(self.handle, float(t0), int(n_macro), y.data_ptr(),
                                 out.data_ptr()))
        return out

    def rk4_step(self, y, out=None, t0=0.0, n_steps=1, h=None):
        """n_steps classical RK4 steps of size h (default: the plan's H) with
        the plan's operator; returns the output tensor."""
        self._bind_stream()
        self._check_state(y)
        if out is None:
            out = torch.empty_like(y)
        self._check_state(out)
        B.check(B.lib().gbs_rk4_step(self.handle, float(t0), int(n_steps),
                                     float(self.H if h is None else h), y.data_ptr(),
                                     out.data_ptr()))
        return out

    def set_sources(self, rhs, flat_index, weight, f0, delay):
        self._bind_stream()
        n = len(rhs)
        B.check(B.lib().gbs_plan_set_sources(self.handle, n, B._arr(ctypes.c_int32, rhs),
                                             B._arr(ctypes.c_int64, flat_index),
                                             B._arr(ctypes.c_double, weight), float(f0),
                                             float(delay)))

    def set_receivers(self, rhs, flat_index):
        """Pressure receivers (right-hand side, index within one field)."""
        self._bind_stream()
        self.n_rec = len(flat_index)
        B.check(B.lib().gbs_plan_set_receivers(self.handle, self.n_rec,
                                               B._arr(ctypes.c_int32, rhs),
                                               B._arr(ctypes.c_int64, flat_index)))

    def step_record(self, y, out=None, t0=0.0, n_macro=1, traces=None):
        """As step(), also returning the receiver traces [n_macro, n_rec]."""
        self._bind_stream()
        self._check_state(y)
        if out is None:
            out = torch.empty_like(y)
        self._check_state(out)
        n_rec = getattr(self, "n_rec", 0)
        if traces is None:
            traces = torch.empty((n_macro, max(n_rec, 1)), dtype=self.dtype, device=self.device)
        B.check(B.lib().gbs_step_record(self.handle, float(t0), int(n_macro), y.data_ptr(),
                                        out.data_ptr(), traces.data_ptr()))
        return out, traces[:, :n_rec]

    def adjoint_workspace(self):
        if getattr(self, "_adj_ws", None) is None:
            nb = ctypes.c_size_t()
            B.check(B.lib().gbs_plan_adjoint_workspace_bytes(self.handle, ctypes.byref(nb)))
            self._adj_ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)
        return self._adj_ws

    def adjoint_step(self, t0, y_in, ybar, trace_bar=None, grad_c2=None):
        """One macro step backwards: ybar (adjoint at t0 + H) is replaced by
        the adjoint at t0; trace_bar [n_rec] is the adjoint of the traces
        recorded at t0 + H; dL/dc^2 is added to grad_c2 (FP64)."""
        self._bind_stream()
        self._check_state(y_in)
        self._check_state(ybar)
        if trace_bar is not None:
            trace_bar = trace_bar.to(self.dtype).contiguous()
        if grad_c2 is not None and (grad_c2.dtype != torch.float64 or not grad_c2.is_contiguous()):
            raise ValueError("grad_c2 must be a contiguous float64 tensor")
        ws = self.adjoint_workspace()
        B.check(B.lib().gbs_adjoint_step(self.handle, float(t0), y_in.data_ptr(), ybar.data_ptr(),
                                         trace_bar.data_ptr() if trace_bar is not None else None,
                                         grad_c2.data_ptr() if grad_c2 is not None else None,
                                         ws.data_ptr(), ws.numel()))
        return ybar

    def pairs_shape(self, n_macro=1):
        """Shape of the buffer gbs_step_keep_pairs fills: [n_macro][k][2] whole
        states (the last two leap-frog levels of every sequence)."""
        return (n_macro, len(self.steps), 2) + self.state_shape

    def step_keep_pairs(self, y, out, pairs, t0=0.0, n_macro=1):
        """As step(), also keeping (y_{N-1}, y_N) of every sequence and macro
        step in ``pairs`` (shape pairs_shape(n_macro), the plan's dtype)."""
        self._bind_stream()
        self._check_state(y)
        self._check_state(out)
        if (pairs.device != self.device or pairs.dtype != self.dtype
                or not pairs.is_contiguous() or tuple(pairs.shape) != self.pairs_shape(n_macro)):
            raise ValueError("pairs must be a contiguous %s tensor of shape %s"
                             % (self.dtype, self.pairs_shape(n_macro)))
        B.check(B.lib().gbs_step_keep_pairs(self.handle, float(t0), int(n_macro), y.data_ptr(),
                                            out.data_ptr(), pairs.data_ptr()))
        return out

    def adjoint_step_pairs(self, t0, y_in, pairs, ybar, trace_bar=None, grad_c2=None):
        """adjoint_step() with the forward levels kept by step_keep_pairs
        (``pairs``: that macro step's [k][2] block) instead of recomputed."""
        self._bind_stream()
        self._check_state(y_in)
        self._check_state(ybar)
        if (pairs.device != self.device or pairs.dtype != self.dtype
                or not pairs.is_contiguous() or tuple(pairs.shape) != self.pairs_shape(1)[1:]):
            raise ValueError("pairs must be one macro step's contiguous block %s"
                             % (self.pairs_shape(1)[1:],))
        if trace_bar is not None:
            trace_bar = trace_bar.to(self.dtype).contiguous()
        if grad_c2 is not None and (grad_c2.dtype != torch.float64 or not grad_c2.is_contiguous()):
            raise ValueError("grad_c2 must be a contiguous float64 tensor")
        ws = self.adjoint_workspace()
        B.check(B.lib().gbs_adjoint_step_pairs(
            self.handle, float(t0), y_in.data_ptr(), pairs.data_ptr(), ybar.data_ptr(),
            trace_bar.data_ptr() if trace_bar is not None else None,
            grad_c2.data_ptr() if grad_c2 is not None else None, ws.data_ptr(), ws.numel()))
        return ybar

    def set_variant(self, variant):
        B.check(B.lib().gbs_plan_set_variant(self.handle, int(variant)))

    def set_form(self, form):
        """GBS_FORM_* flags of the blocked passes (gbs_plan_set_form)."""
        B.check(B.lib().gbs_plan_set_form(self.handle, int(form)))

    def set_wave_order(self, order):
        """Workgroup order of the blocked passes (gbs_plan_set_wave_order)."""
        B.check(B.lib().gbs_plan_set_wave_order(self.handle, int(order)))

    def autotune(self, y, out=None, macro_steps=5, lanes=0):
        """Times the blocked variants, bands and lane counts
        (gbs_plan_autotune) from ``y`` into ``out`` (a scratch copy if None)
        and keeps the fastest; ``lanes`` > 0 fixes the lane count.  Returns
        (variant, band, lanes)."""
        self._bind_stream()
        self._check_state(y)
        scratch = y.clone() if out is None else out
        self._check_state(scratch)
        v, b, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(int(lanes))
        B.check(B.lib().gbs_plan_autotune(self.handle, y.data_ptr(), scratch.data_ptr(),
                                          int(macro_steps), ctypes.byref(v), ctypes.byref(b),
                                          ctypes.byref(l)))
        self.lanes = l.value
        return v.value, b.value, l.value

    def set_lanes(self, lanes):
        """Streams the blocked passes of a macro step are spread over (1..4)."""
        B.check(B.lib().gbs_plan_set_lanes(self.handle, int(lanes)))
        self.lanes = int(lanes)

    def autotune_adjoint(self, y, repeats=4):
        """Times the blocked adjoint from kept levels (adjoint_step_pairs) on
        1, 2 and 3 lanes from the state ``y`` and keeps the fastest count in
        ``adjoint_lanes`` (the forward's lane count is left as it was).
        Returns it, or None when the plan's adjoint is not the blocked one."""
        self._bind_stream()
        if not self.blocked_adjoint():
            return None
        self._check_state(y)
        fwd = self.lanes
        pairs = torch.empty(self.pairs_shape(1), dtype=self.dtype, device=self.device)
        self.step_keep_pairs(y, torch.empty_like(y), pairs)
        ybar = torch.zeros_like(y)
        grad = (torch.zeros(self.c2_field.shape, dtype=torch.float64, device=self.device)
                if self.c2_field is not None else None)
        best, best_t = fwd, None
        for lanes in (1, 2, 3):
            self.set_lanes(lanes)
            self.adjoint_step_pairs(0.0, y, pairs[0], ybar, grad_c2=grad)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(self.stream)
            for _ in range(repeats):
                self.adjoint_step_pairs(0.0, y, pairs[0], ybar, grad_c2=grad)
            b.record(self.stream)
            b.synchronize()
            t = a.elapsed_time(b)
            if best_t is None or t < best_t * 0.98:
                best, best_t = lanes, t
        self.set_lanes(fwd)
        self.adjoint_lanes = best
        return best

    def variant(self):
        out = ctypes.c_int32()
        B.check(B.lib().gbs_plan_get_variant(self.handle, ctypes.byref(out)))
        return out.value

    def blocked_adjoint(self):
        """Whether gbs_adjoint_step takes the temporally blocked form (2-D
        FD4 with a temporally blocked forward variant), the one that can use
        kept pairs."""
        return (self.op == B.ACOUSTIC2D and self.problem.fd_order == 4
                and self.variant() in _TEMPORAL)

    def set_timing(self, on):
        """on: bool, or the number of macro steps to create events for."""
        B.check(B.lib().gbs_plan_set_timing(self.handle, int(on)))

    def get_timing(self):
        """(leap-frog ms, launches, first-evaluation ms, launches) since the
        last read."""
        a, b = ctypes.c_double(), ctypes.c_int64()
        c, d = ctypes.c_double(), ctypes.c_int64()
        B.check(B.lib().gbs_plan_get_timing(self.handle, ctypes.byref(a), ctypes.byref(b),
                                            ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def get_adjoint_timing(self):
        """(blocked adjoint pass ms, launches, their algorithmic bytes) since
        the last read (timing on, one lane)."""
        a, b, c = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        B.check(B.lib().gbs_plan_get_adjoint_timing(self.handle, ctypes.byref(a), ctypes.byref(b),
                                                    ctypes.byref(c)))
        return a.value, b.value, c.value

    def algorithmic_bytes(self):
        """(stepping-kernel bytes, launches, auxiliary bytes, launches) per
        macro step, for the variant in use."""
        a, b = ctypes.c_double(), ctypes.c_int64()
        c, d = ctypes.c_double(), ctypes.c_int64()
        B.check(B.lib().gbs_plan_algorithmic_bytes(self.handle, ctypes.byref(a), ctypes.byref(b),
                                                   ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def updates_per_macro_step(self):
        out = ctypes.c_double()
        B.check(B.lib().gbs_plan_updates_per_macro_step(self.handle, ctypes.byref(out)))
        return out.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                B.lib().gbs_plan_destroy(h)
            except Exception:
                pass
            self.handle = None


class GBSBatch:
    """Many independent 2-D acoustic instances (own grid, c^2 field or
    constant, H) advanced together: one launch per pass round for the whole
    batch, optionally replayed from a captured hipGraph.

    instances: list of dicts with keys n = (nx, ny), H, and either c2 (float)
    or c2_field (tensor [ny][nx]) with optional c_max."""

    def __init__(self, instances, p, steps, w, fd_order=4, dtype=torch.float64, device="cuda",
                 check_stability=True):
        if not torch.cuda.is_available():
            raise RuntimeError("GBSBatch needs a HIP device; there is no CPU path")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dtype = dtype
        flags = 0 if check_stability else B.FLAG_NO_STABILITY_CHECK
        self.fields = []
        probs = (B.Problem * len(instances))()
        Hs = (ctypes.c_double * len(instances))()
        self.shapes = []
        for i, inst in enumerate(instances):
            nx, ny = inst["n"]
            ptr, c_max = None, 0.0
            if inst.get("c2_field") is not None:
                f = inst["c2_field"].to(device=self.device, dtype=dtype).contiguous()
                self.fields.append(f)
                ptr = f.data_ptr()
                c_max = inst.get("c_max") or float(f.max().sqrt())
            probs[i] = B.make_problem(B.ACOUSTIC2D, (nx, ny), fd_order, 1, _DT[dtype],
                                      inst.get("c2", 1.0), ptr, c_max, flags)
            Hs[i] = float(inst["H"])
            self.shapes.append((1, 3, ny, nx))
        self._probs, self._Hs = probs, Hs
        self.scheme = B.make_scheme(p, steps, w)
        nb = ctypes.c_size_t()
        B.check(B.lib().gbs_batch_workspace_bytes(len(instances), probs, ctypes.byref(self.scheme),
                                                  ctypes.byref(nb)))
        self.workspace = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.handle = ctypes.c_void_p()
        B.check(B.lib().gbs_batch_plan_create(ctypes.byref(self.handle), len(instances), probs,
                                              ctypes.byref(self.scheme), Hs,
                                              self.workspace.data_ptr(), self.workspace.numel(),
                                              self.stream.cuda_stream))

    def _bind_stream(self):
        """Enqueue on torch's current stream of the plan's device."""
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            B.check(B.lib().gbs_batch_set_stream(self.handle, cur.cuda_stream))
            self.stream = cur

    def _ptrs(self, states):
        self._bind_stream()
        if len(states) != len(self.shapes):
            raise ValueError("need one state per instance")
        for s, shp in zip(states, self.shapes):
            if (s.device != self.device or s.dtype != self.dtype or not s.is_contiguous()
                    or s.numel() != int(torch.Size(shp).numel())):
                raise ValueError("state must be a contiguous %s tensor of %s elements on %s"
                                 % (self.dtype, shp, self.device))
        return (ctypes.c_void_p * len(states))(*[s.data_ptr() for s in states])

    def step(self, states, n_macro=1):
        """n_macro macro steps of every instance, in place."""
        B.check(B.lib().gbs_batch_step(self.handle, int(n_macro), self._ptrs(states)))
        return states

    def set_variant(self, variant=0, band=0):
        B.check(B.lib().gbs_batch_set_variant(self.handle, int(variant), int(band)))

    def set_graph(self, on):
        B.check(B.lib().gbs_batch_set_graph(self.handle, 1 if on else 0))

    def autotune(self, states, macro_steps=2):
        """Times the candidate kernels on ``states`` (which are advanced) and
        keeps the fastest; returns (variant, band)."""
        v, b = ctypes.c_int32(), ctypes.c_int32()
        B.check(B.lib().gbs_batch_autotune(self.handle, self._ptrs(states), int(macro_steps),
                                           ctypes.byref(v), ctypes.byref(b)))
        return v.value, b.value

    def updates_per_macro_step(self):
        out = ctypes.c_double()
        B.check(B.lib().gbs_batch_updates_per_macro_step(self.handle, ctypes.byref(out)))
        return out.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                B.lib().gbs_batch_plan_destroy(h)
            except Exception:
                pass
            self.handle = None
