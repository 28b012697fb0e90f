"""ctypes binding of libgbs.so (the C ABI declared in include/gbs.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory (states, workspace) and the HIP
stream.  There is no CPU fallback: without the built library, or without a
GPU, the calls that launch kernels raise.
"""
import ctypes
import os
import re

from . import build as _build

GBS_OK, GBS_EINVAL, GBS_ESTEPS, GBS_EORDER = 0, -1, -2, -3
GBS_ESINGULAR, GBS_EUNSTABLE, GBS_EDEVICE, GBS_ENOMEM, GBS_EUNSUPPORTED = -4, -5, -6, -7, -8
ADVECT1D, ACOUSTIC2D, ACOUSTIC3D = 1, 2, 3
FD_SPECTRAL = 0                 # fd_order of the Fourier derivative (ADVECT1D)
F32, F64 = 1, 2
FLAG_NO_STABILITY_CHECK = 1
VARIANT_AUTO, VARIANT_FLAT, VARIANT_MARCH8, VARIANT_MARCH16 = 0, 1, 2, 3
VARIANT_MARCH8_NT, VARIANT_MARCH16_NT = 4, 5
VARIANT_TEMPORAL, VARIANT_TEMPORAL4, VARIANT_TEMPORAL_S5, VARIANT_TEMPORAL_S6 = 6, 7, 8, 9
VARIANT_PLAIN = 10
VARIANT_TEMPORAL_WG4, VARIANT_TEMPORAL_WG8 = 11, 12
VARIANT_TILE3D = 13
FORM_SHARED_F0, FORM_FUSED_COMBINE, FORM_ALIGNED_FIRST = 1, 2, 4
MAX_SEQ = 16
MAX_SRC = 16
MAX_REC = 1024

_NAMES = {GBS_EINVAL: "EINVAL", GBS_ESTEPS: "ESTEPS", GBS_EORDER: "EORDER",
          GBS_ESINGULAR: "ESINGULAR", GBS_EUNSTABLE: "EUNSTABLE", GBS_EDEVICE: "EDEVICE",
          GBS_ENOMEM: "ENOMEM", GBS_EUNSUPPORTED: "EUNSUPPORTED"}


class GBSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(status, "?"), status, msg))
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("fd_order", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("n_rhs", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("c2", ctypes.c_double), ("c2_field", ctypes.c_void_p), ("c_max", ctypes.c_double),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Scheme(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("k", ctypes.c_int32),
                ("steps", ctypes.POINTER(ctypes.c_int32)),
                ("weights", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib_path():
    return _build.LIB


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        path = lib_path()
        if not os.path.exists(path):
            raise RuntimeError("%s is missing: build it with `python -m paper_1907_11771_amd.build`"
                               % path)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        i32, i64, dbl, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
        sig = {
            "gbs_weights": [i32, i32, P(i32), i32, P(i32), P(i64), P(i64), P(dbl), P(dbl)],
            "gbs_isb": [i32, P(i32), P(dbl), P(dbl)],
            "gbs_plan_workspace_bytes": [P(Problem), P(Scheme), P(sz)],
            "gbs_plan_create": [P(vp), P(Problem), P(Scheme), dbl, vp, sz, vp],
            "gbs_plan_set_sources": [vp, i32, P(i32), P(i64), P(dbl), dbl, dbl],
            "gbs_step": [vp, dbl, i32, vp, vp],
            "gbs_rk4_step": [vp, dbl, i32, dbl, vp, vp],
            "gbs_plan_set_timing": [vp, i32],
            "gbs_plan_set_variant": [vp, i32],
            "gbs_plan_get_variant": [vp, P(i32)],
            "gbs_plan_autotune": [vp, vp, vp, i32, P(i32), P(i32), P(i32)],
            "gbs_plan_set_lanes": [vp, i32],
            "gbs_plan_set_band": [vp, i32],
            "gbs_plan_set_wave_order": [vp, i32],
            "gbs_plan_set_form": [vp, i32],
            "gbs_plan_set_stream": [vp, vp],
            "gbs_plan_get_timing": [vp, P(dbl), P(i64), P(dbl), P(i64)],
            "gbs_plan_get_adjoint_timing": [vp, P(dbl), P(i64), P(dbl)],
            "gbs_plan_updates_per_macro_step": [vp, P(dbl)],
            "gbs_plan_algorithmic_bytes": [vp, P(dbl), P(i64), P(dbl), P(i64)],
            "gbs_plan_destroy": [vp],
            "gbs_plan_set_receivers": [vp, i32, P(i32), P(i64)],
            "gbs_step_record": [vp, dbl, i32, vp, vp, vp],
            "gbs_plan_adjoint_workspace_bytes": [vp, P(sz)],
            "gbs_adjoint_step": [vp, dbl, vp, vp, vp, vp, vp, sz],
            "gbs_step_keep_pairs": [vp, dbl, i32, vp, vp, vp],
            "gbs_adjoint_step_pairs": [vp, dbl, vp, vp, vp, vp, vp, vp, sz],
            "gbs_batch_workspace_bytes": [i32, P(Problem), P(Scheme), P(sz)],
            "gbs_batch_plan_create": [P(vp), i32, P(Problem), P(Scheme), P(dbl), vp, sz, vp],
            "gbs_batch_set_variant": [vp, i32, i32],
            "gbs_batch_set_graph": [vp, i32],
            "gbs_batch_set_stream": [vp, vp],
            "gbs_batch_step": [vp, i32, P(vp)],
            "gbs_batch_autotune": [vp, P(vp), i32, P(i32), P(i32)],
            "gbs_batch_updates_per_macro_step": [vp, P(dbl)],
            "gbs_batch_plan_destroy": [vp],
            "gbs_step_scratch": [P(Problem), P(Scheme), dbl, dbl, i32, vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.gbs_last_error.argtypes = []
        L.gbs_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_symbols():
    """Function names declared in include/gbs.h."""
    path = os.path.join(_build.ROOT, "include", "gbs.h")
    with open(path) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gbs_\w+)\s*\(", text, re.M)))


def check(status):
    if status != GBS_OK:
        raise GBSError(status, lib().gbs_last_error().decode())
    return status


def _arr(ctype, vals):
    vals = list(vals)
    return (ctype * max(len(vals), 1))(*vals)


def weights(p, steps, free_idx=(), c_free=()):
    """Weights (FP64, nearest) and the exact-R ISB.  c_free: (num, den) pairs."""
    m = len(steps)
    out = (ctypes.c_double * m)()
    isb = ctypes.c_double()
    nums = [int(a) for a, _ in c_free]
    dens = [int(b) for _, b in c_free]
    check(lib().gbs_weights(p, m, _arr(ctypes.c_int32, steps), len(free_idx),
                            _arr(ctypes.c_int32, free_idx), _arr(ctypes.c_int64, nums),
                            _arr(ctypes.c_int64, dens), out, ctypes.byref(isb)))
    return list(out), isb.value


def isb(steps, w):
    out = ctypes.c_double()
    check(lib().gbs_isb(len(steps), _arr(ctypes.c_int32, steps), _arr(ctypes.c_double, w),
                        ctypes.byref(out)))
    return out.value


def make_problem(op, n, fd_order=4, n_rhs=1, dtype=F64, c2=1.0, c2_field_ptr=None, c_max=0.0,
                 flags=0):
    pr = Problem()
    pr.op, pr.fd_order, pr.n_rhs, pr.dtype = op, fd_order, n_rhs, dtype
    nn = list(n) + [1] * (3 - len(n))
    for a in range(3):
        pr.n[a] = int(nn[a])
    pr.c2 = float(c2)
    pr.c2_field = c2_field_ptr
    pr.c_max = float(c_max)
    pr.flags = flags
    return pr


def make_scheme(p, steps, w):
    sc = Scheme()
    sc.p, sc.k = p, len(steps)
    sc._steps = _arr(ctypes.c_int32, steps)      # keep alive
    sc._w = _arr(ctypes.c_double, w)
    sc.steps = ctypes.cast(sc._steps, ctypes.POINTER(ctypes.c_int32))
    sc.weights = ctypes.cast(sc._w, ctypes.POINTER(ctypes.c_double))
    return sc


def workspace_bytes(problem, scheme):
    out = ctypes.c_size_t()
    check(lib().gbs_plan_workspace_bytes(ctypes.byref(problem), ctypes.byref(scheme),
                                         ctypes.byref(out)))
    return out.value


def plan_create(problem, scheme, H, workspace_ptr, workspace_bytes_, stream_ptr=None):
    handle = ctypes.c_void_p()
    check(lib().gbs_plan_create(ctypes.byref(handle), ctypes.byref(problem), ctypes.byref(scheme),
                                float(H), workspace_ptr, workspace_bytes_, stream_ptr))
    return handle


def plan_destroy(handle):
    if handle:
        check(lib().gbs_plan_destroy(handle))
