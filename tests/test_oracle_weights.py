"""Pins for oracle.weights: printed weights, closed forms, order conditions."""
from fractions import Fraction

import pytest

from oracle import stability as S
from oracle import weights as W
from synth import schemes
from tests.conftest import golden_lines


def test_table1_printed_weights_exact():
    # Sect. 3.3: the exact weights printed for the order-8 and order-12 schemes
    for line in golden_lines("paper_table1_weights.txt"):
        order, steps, ws = [x.strip() for x in line.split("|")]
        steps = [int(x) for x in steps.split()]
        want = [Fraction(x) for x in ws.split()]
        assert W.weights(int(order), steps) == want


def test_square_order4_closed_form():
    # Richardson over N = {2, 4}: c = (-1/3, 4/3)
    assert W.weights(4, [2, 4]) == [Fraction(-1, 3), Fraction(4, 3)]


@pytest.mark.parametrize("steps", [[2, 4], [2, 4, 6], [2, 4, 6, 8], [2, 16, 18, 20],
                                   [4, 10, 2, 8, 6]])
def test_square_matches_lagrange_closed_form(steps):
    p = 2 * len(steps)
    assert W.weights(p, steps) == W.weights_square_closed_form(steps)


@pytest.mark.parametrize("sch", schemes.ALL, ids=lambda s: s["name"])
def test_order_conditions_via_taylor(sch):
    # Order p means R(xi) = exp(xi) + O(xi^{p+1}) (App. A / Sect. 3.2): the
    # first p+1 Taylor coefficients of sum c_i P_i equal 1/k!, with P_i built
    # from the GBS recurrence, independently of the Vandermonde matrix.
    c = W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    r = S.extrapolated_poly(sch["steps"], c)
    e = S.taylor_errors(r, sch["p"] + 2)
    assert all(x == 0 for x in e[: sch["p"] + 1])
    assert e[sch["p"] + 1] != 0 or e[sch["p"] + 2] != 0   # not of higher order by accident


def test_dep_free_split_is_a_reparametrisation():
    # eq. (cdep_computation): any choice of free columns describes the same
    # affine family; feeding the full vector back with another free set
    # returns it unchanged.
    sch = schemes.GBS_8_6
    c = W.weights(8, sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    other_free = [0, 2, 5, 6, 8, 9, 10]
    c2 = W.weights(8, sch["steps"], other_free, [c[i] for i in other_free])
    assert c2 == c


def test_weights_sum_to_one_and_match_vandermonde_rows():
    sch = schemes.ORDER8_K6
    c = W.weights(8, sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    assert sum(c) == 1
    v = W.vandermonde(8, sch["steps"])
    for k, row in enumerate(v):
        assert sum(a * b for a, b in zip(row, c)) == (1 if k == 0 else 0)


def test_rejects_bad_steps():
    with pytest.raises(ValueError):
        W.weights(4, [2, 3])
    with pytest.raises(ValueError):
        W.weights(4, [2, 2])
    with pytest.raises(ValueError):
        W.weights(8, [2, 4, 6])           # fewer than p/2 sequences


def test_fp64_rounding_is_nearest():
    c = W.weights(8, [2, 16, 18, 20])
    for x, d in zip(c, W.to_fp64(c)):
        err = abs(Fraction(d) - x)
        # the neighbours of d are farther from x
        import math
        up = Fraction(math.nextafter(d, math.inf))
        dn = Fraction(math.nextafter(d, -math.inf))
        assert err <= abs(up - x) and err <= abs(dn - x)
