"""Pins for oracle.optimize: the paper's printed optimal ISB_n values, and
the frozen configuration scheme."""
import json
import os
from fractions import Fraction

import pytest

from oracle import optimize as O
from oracle import stability as S
from oracle import weights as W
from synth import schemes
from tests.conftest import GOLDEN, golden_lines


@pytest.mark.parametrize("line", golden_lines("paper_optimum_isb_n.txt"))
def test_optimiser_reproduces_printed_optimum(line):
    order, nmax, dep, val = [x.strip() for x in line.split("|")]
    order, nmax = int(order), int(nmax)
    dep = [int(x) for x in dep.split()]
    free = [n for n in range(2, nmax + 1, 2) if n not in dep]
    steps = dep + free
    y, cf = O.optimise(order, steps, list(range(len(dep), len(steps))), tol=1e-3,
                       n_samples=400, n_gon=64)
    assert cf is not None
    assert abs(y / (nmax + 1) - float(val)) < 3e-4


def test_frozen_scheme_matches_golden_and_inputs():
    with open(os.path.join(GOLDEN, "order8_k6_scheme.json")) as fh:
        g = json.load(fh)
    sch = schemes.ORDER8_K6
    assert tuple(g["steps"]) == sch["steps"] and tuple(g["free_idx"]) == sch["free_idx"]
    assert tuple(g["c_free"]) == sch["c_free"]
    c = W.weights(8, sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    isb = S.isb(S.extrapolated_poly(sch["steps"], c))
    assert isb == pytest.approx(g["exact_isb"], rel=1e-12)
    # accepted when within 1% of the optimiser's (tangency-limited) optimum
    assert isb >= 0.99 * g["lp_isb"]


@pytest.mark.slow
def test_freeze_script_reproduces_golden():
    from oracle import freeze_scheme
    with open(os.path.join(GOLDEN, "order8_k6_scheme.json")) as fh:
        g = json.load(fh)
    out = freeze_scheme.freeze()
    assert out["c_free"] == g["c_free"]
