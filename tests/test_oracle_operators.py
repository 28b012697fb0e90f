"""Pins for oracle.operators: stencil weights by polynomial exactness,
skew-symmetry, convergence order, adjoint by the dot-product identity."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import operators as OP
from synth import fields


def test_fd4_and_fd8_weights():
    assert OP.centred_first_derivative_weights(2) == [Fraction(2, 3), Fraction(-1, 12)]
    assert OP.centred_first_derivative_weights(4) == [Fraction(4, 5), Fraction(-1, 5),
                                                      Fraction(4, 105), Fraction(-1, 280)]


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_polynomial_exactness(r):
    # exact (to rounding) for degree <= 2r at points whose stencil does not wrap
    # (a coarse grid, dx = 1/2, so that the degree 2r+1 error is O(1))
    m = 24
    dx = 0.5
    x = np.arange(m) * dx - 5.3
    interior = slice(r, m - r)
    for deg in range(0, 2 * r + 2):
        u = x ** deg
        du = deg * x ** (deg - 1) if deg else np.zeros(m)
        scale = max(1.0, np.max(np.abs(du)))
        err = np.max(np.abs(OP.d1(u, 0, dx, r)[interior] - du[interior]))
        if deg <= 2 * r:
            assert err / scale < 1e-12, (r, deg, err)
        else:
            assert err > 1e-3, (r, deg, err)     # truncation error dx^{2r} u^{(2r+1)} ~ O(1)


@pytest.mark.parametrize("r,order", [(2, 4), (4, 8)])
def test_convergence_order(r, order):
    errs = []
    for m in (32, 64):
        x = np.arange(m) / m
        u = np.sin(2 * np.pi * 3 * x)
        du = 2 * np.pi * 3 * np.cos(2 * np.pi * 3 * x)
        errs.append(np.max(np.abs(OP.d1(u, 0, 1.0 / m, r) - du)))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - order) < 0.3


def test_skew_symmetry():
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal((2, 40))
    for r in (2, 4):
        a = np.dot(OP.d1(u, 0, 0.1, r), v)
        b = -np.dot(u, OP.d1(v, 0, 0.1, r))
        assert a == pytest.approx(b, rel=1e-12)


@pytest.mark.parametrize("shape,r", [((12, 16), 2), ((6, 8, 10), 4)])
def test_acoustic_transpose(shape, r):
    rng = np.random.default_rng(2)
    c2 = fields.lognormal_speed(shape, seed=3) ** 2
    op = OP.Acoustic(shape, c2=c2, r=r)
    d = len(shape)
    u = rng.standard_normal((1 + d,) + shape)
    w = rng.standard_normal((1 + d,) + shape)
    lhs = np.sum(op.linear(u) * w)
    rhs = np.sum(u * op.matvec_T(w))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_acoustic_plane_wave_dispersion():
    # a plane wave along x: p = cos(2 pi k x), v_x = cos(2 pi k x) travels at
    # speed c: f = -c * d/dx (p, vx) for c = 1, to FD4 accuracy
    n = 128
    x = np.arange(n) / n
    k = 2
    y = np.zeros((3, n, n))
    y[0] = np.cos(2 * np.pi * k * x)[None, :]
    y[1] = y[0]
    f = OP.Acoustic((n, n), c2=1.0, r=2)(0.0, y)
    want = 2 * np.pi * k * np.sin(2 * np.pi * k * x)[None, :]
    assert np.max(np.abs(f[0] - want)) < 2e-3 * 2 * np.pi * k
    assert np.max(np.abs(f[1] - want)) < 2e-3 * 2 * np.pi * k
    assert np.max(np.abs(f[2])) == 0.0


@pytest.mark.parametrize("f0,delay", [(25.0, 0.06), (3.0, 0.5)])
def test_ricker_amplitude_closed_form_points(f0, delay):
    # the Ricker wavelet r(tau) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2),
    # tau = t - delay: r = 1 at the delay, zeros at tau = +-1/(sqrt 2 pi f0),
    # minima -2 exp(-3/2) at tau = +-sqrt(3/2)/(pi f0), even in tau, and
    # decaying to 0 (a factor of 2 in either exponent, a wrong sign or a
    # shifted delay moves one of these points)
    s = OP.Source((0, 0), f0, delay, 1.0)
    assert s.amplitude(delay) == 1.0
    tz = 1.0 / (np.sqrt(2.0) * np.pi * f0)
    tm = np.sqrt(1.5) / (np.pi * f0)
    for sign in (1.0, -1.0):
        assert abs(s.amplitude(delay + sign * tz)) <= 1e-14
        assert s.amplitude(delay + sign * tm) == pytest.approx(-2.0 * np.exp(-1.5), rel=1e-14)
        # a minimum: neighbours on both sides are larger
        for d in (1e-4, -1e-4):
            assert s.amplitude(delay + sign * tm * (1 + d)) > s.amplitude(delay + sign * tm)
    taus = np.linspace(0.0, 3.0 * tm, 50)
    assert np.allclose(s.amplitude(delay + taus), s.amplitude(delay - taus), rtol=0, atol=1e-12)
    assert abs(s.amplitude(delay + 6.0 / f0)) < 1e-100
