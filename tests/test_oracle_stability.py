"""Pins for oracle.stability: closed form on the imaginary axis, printed
ISB_n values, the RK4 textbook value, the order (mod 4) rule."""
import math
from fractions import Fraction

import mpmath
import pytest

from oracle import stability as S
from oracle import weights as W
from synth import schemes
from tests.conftest import golden_lines

BY_NAME = {s["name"]: s for s in schemes.ALL}


def _c(sch):
    return W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])


@pytest.mark.parametrize("n", [2, 4, 12, 30])
@pytest.mark.parametrize("theta", ["0.1", "0.7", "0.999", "1.3", "2.5"])
def test_poly_matches_imaginary_axis_closed_form(n, theta):
    mpmath.mp.dps = 60
    th = mpmath.mpf(theta)
    coeffs = S.gbs_poly(n)
    xi = mpmath.mpc(0, n * th)
    rec = S.poly_eval([mpmath.mpf(q.numerator) / q.denominator for q in coeffs], xi)
    cf = S.gbs_poly_imag_closed_form(n, th)
    assert abs(rec - cf) <= mpmath.mpf(10) ** -40 * max(1, abs(cf))


def test_poly_degree_and_low_order():
    # N+1 function evaluations give degree N+1; the unextrapolated step is
    # second order: P_N = 1 + xi + xi^2/2 + O(xi^3)
    for n in (2, 4, 10):
        p = S.gbs_poly(n)
        assert len(p) == n + 2 and p[-1] != 0
        assert p[:3] == [1, 1, Fraction(1, 2)]
        assert p[3] != Fraction(1, 6)


@pytest.mark.parametrize("line", golden_lines("paper_isb_n.txt"))
def test_printed_isb_n(line):
    name, val, _src = [x.strip() for x in line.split("|")]
    sch = BY_NAME[name]
    r = S.extrapolated_poly(sch["steps"], _c(sch))
    got = S.isb_n(sch["steps"], r)
    # the paper rounds some values and truncates others to four decimals
    shown = {round(got, 4), math.floor(got * 1e4) / 1e4}
    assert any(abs(float(val) - x) < 1e-12 for x in shown), (name, got)


def test_rk4_isb_textbook():
    want = float(golden_lines("rk4_isb.txt")[0])
    got = S.isb(S.rk4_poly())
    assert got == pytest.approx(2 * math.sqrt(2), rel=1e-14)
    assert round(got, 4) == want


@pytest.mark.parametrize("p,steps", [(6, [2, 4, 6]), (10, [2, 4, 6, 8, 10]), (6, [2, 8, 12])])
def test_order_2_mod_4_has_no_isb(p, steps):
    # Sect. 2.2: orders 6, 10, 14, ... have ISB = 0
    assert S.isb(S.extrapolated_poly(steps, W.weights(p, steps))) == 0.0


def test_isb_brute_force_for_config_scheme():
    # dense sampling of |R(iy)| in high precision: <= 1 up to the ISB, > 1 just past it
    mpmath.mp.dps = 40
    sch = schemes.ORDER8_K6
    r = S.extrapolated_poly(sch["steps"], _c(sch))
    isb = S.isb(r)
    rm = [mpmath.mpf(x.numerator) / x.denominator for x in r]
    for k in range(1, 401):
        y = mpmath.mpf(isb) * k / 400 * (1 - mpmath.mpf(10) ** -9)
        assert abs(S.poly_eval(rm, mpmath.mpc(0, y))) <= 1 + mpmath.mpf(10) ** -30
    y = mpmath.mpf(isb) * (1 + mpmath.mpf(10) ** -6)
    assert abs(S.poly_eval(rm, mpmath.mpc(0, y))) > 1


def test_square_order4_isb():
    r = S.extrapolated_poly([2, 4], W.weights(4, [2, 4]))
    # leading even-part error terms: e5 = -1/320, e6 = -1/720 (exact Taylor)
    e = S.taylor_errors(r, 6)
    assert e[5] == Fraction(-1, 320) and e[6] == Fraction(-1, 720)
    assert S.isb(r) == pytest.approx(3.3635857, abs=5e-7)
