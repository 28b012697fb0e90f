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


def rel_err(got, want):
    """max |got - want| / max |want| (per whole array)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))
