"""Helpers for the GPU parity tests: run the library and the oracle on the
same seeded inputs."""
from fractions import Fraction

import numpy as np
import torch

from oracle import weights as W
from paper_1907_11771_amd import binding as B
from paper_1907_11771_amd.plan import GBSPlan, scheme_weights


def oracle_weights(sch):
    c = W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    return list(sch["steps"]), W.to_fp64(c)


def lib_plan(op, n, sch, H, **kw):
    steps, w, _ = scheme_weights(sch)
    return GBSPlan(op, n, sch["p"], steps, w, H, **kw)


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def rel_err(got, want, field_axis):
    """The parity norm, per field: for every field q (the slices along
    ``field_axis``, the axis that indexes p, v_x, v_y[, v_z] or u),
    max |got_q - want_q| / max |want_q|, and the largest of these.
    field_axis=None: the array is one field (a c^2 gradient, one field of a
    state).  Every caller names the axis, so that a small field (a velocity
    that starts at zero) is not measured against a larger one."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    if field_axis is None:
        got, want = got[None], want[None]
        field_axis = 0
    got = np.moveaxis(got, field_axis, 0)
    want = np.moveaxis(want, field_axis, 0)
    errs = []
    for q in range(want.shape[0]):
        scale = np.max(np.abs(want[q]))
        assert scale > 0, "field %d of the reference is zero" % q
        errs.append(float(np.max(np.abs(got[q] - want[q])) / scale))
    return max(errs)
