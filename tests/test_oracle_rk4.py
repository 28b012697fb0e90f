"""The RK4 comparison method of the oracle (App. A) against what fixes it
independently: one step on y' = lambda y is the degree-4 Taylor polynomial
of exp; its imaginary stability boundary is the printed 2.8284 (2 sqrt 2);
on the constant-c acoustic system it equals the Fourier closed form; it
converges at order 4 to the semi-discrete solution exp(tA) y0, which in turn
is what the GBS closed form approaches as H -> 0."""
import math

import numpy as np
import pytest

from oracle import gbs as G
from oracle import operators as OP
from oracle import rk4 as RK
from oracle import spectral as SP
from oracle import weights as W
from synth import fields, schemes
from tests.conftest import golden_lines


def test_one_step_is_the_taylor_polynomial():
    for lam in (0.7j, -0.3 + 1.1j, 2.5j):
        for h in (0.1, 0.9):
            got = RK.rk4_step(lambda t, y: lam * y, 0.0, np.array([1.0 + 0j]), h)[0]
            z = h * lam
            want = sum(z ** k / math.factorial(k) for k in range(5))
            assert abs(got - want) <= 1e-15 * abs(want)


def test_imaginary_stability_boundary_is_the_printed_value():
    isb = float(golden_lines("rk4_isb.txt")[0])
    r = lambda y: abs(SP.rk4_amplification(np.array([1j * y]), 1.0, 1)[0])
    assert r(isb) <= 1.0 + 1e-12                    # printed value rounds 2 sqrt 2 down
    assert r(2 * math.sqrt(2) * (1 + 1e-6)) > 1.0
    assert all(r(y) <= 1.0 + 1e-15 for y in np.linspace(0, 2 * math.sqrt(2), 200))


def test_acoustic_steps_match_the_fourier_closed_form():
    n = 24
    y0 = fields.acoustic2d_pulse_modes(n, n_modes=5, kmax=4, width=0.1, seed=3)
    op = OP.Acoustic((n, n), c2=1.3, r=2)
    h = 0.8 * 2 * math.sqrt(2) / (math.sqrt(1.3) * 1.3722220 * n * math.sqrt(2))
    got = RK.integrate(op, 0.0, y0, h, 5)
    want = SP.acoustic_rk4(y0, 1.3, h, 5)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_converges_at_order_four_to_the_semi_discrete_solution():
    n = 32
    y0 = fields.acoustic2d_pulse_modes(n, n_modes=6, kmax=5, width=0.1, seed=4)
    t = 0.05
    exact = SP.acoustic_exact(y0, 1.0, t)
    errs = []
    for m in (10, 20, 40):
        errs.append(np.max(np.abs(SP.acoustic_rk4(y0, 1.0, t / m, m) - exact)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.7 < q < 4.3 for q in rates), rates


def test_gbs_closed_form_approaches_the_semi_discrete_solution():
    # the same exact reference the time-to-solution comparison uses
    n = 32
    sch = schemes.ORDER8_K6
    steps = list(sch["steps"])
    from fractions import Fraction
    c = W.to_fp64(W.weights(sch["p"], steps, sch["free_idx"], [Fraction(x) for x in sch["c_free"]]))
    y0 = fields.acoustic2d_pulse_modes(n, n_modes=6, kmax=5, width=0.1, seed=4)
    t = 0.2
    exact = SP.acoustic_exact(y0, 1.0, t)
    errs = [np.max(np.abs(SP.acoustic(y0, 1.0, t / m, steps, c, m) - exact)) for m in (4, 8)]
    assert errs[1] < errs[0] / 100                  # order 8: 2^8 = 256 in the limit
    # and the literal oracle agrees with its closed form here
    lit = G.integrate(OP.Acoustic((n, n), c2=1.0, r=2), 0.0, y0, t / 8, 8, steps, c)
    assert np.max(np.abs(lit - SP.acoustic(y0, 1.0, t / 8, steps, c, 8))) <= 1e-12
