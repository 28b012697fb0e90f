"""Pins for oracle.gbs and oracle.spectral: closed forms on y' = i w y,
convergence orders (also with explicit time dependence), brute-force matrix
powers on tiny grids, agreement of the two oracles, and the energy bound for
variable coefficients."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import gbs as G
from oracle import operators as OP
from oracle import spectral as SP
from oracle import stability as S
from oracle import weights as W
from synth import fields, schemes, workloads


def _cf(sch):
    c = W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    return list(sch["steps"]), W.to_fp64(c)


@pytest.mark.parametrize("sch", [schemes.SQUARE4_2_4, schemes.ORDER8_K6, schemes.GBS_8_6],
                         ids=lambda s: s["name"])
@pytest.mark.parametrize("wH", [0.3, 1.7, 5.5])
def test_scalar_imaginary_matches_closed_form(sch, wH):
    steps, c = _cf(sch)
    w = 3.0
    H = wH / w
    got = G.macro_step(lambda t, y: 1j * w * y, 0.0, np.array([1.0 + 0j]), H, steps, c)[0]
    want = sum(ci * S.gbs_poly_imag_closed_form(n, complex(wH / n)) for n, ci in zip(steps, c))
    assert abs(got - want) < 1e-13 * max(1.0, abs(want))


def test_function_evaluation_count():
    steps, c = _cf(schemes.ORDER8_K6)
    calls = []

    def f(t, y):
        calls.append(t)
        return -y

    G.macro_step(f, 0.0, np.ones(3), 0.1, steps, c)
    assert len(calls) == 1 + sum(steps) == 43
    assert calls.count(0.0) == 1                       # f(t0, y0) shared by all sequences


@pytest.mark.parametrize("sch,order", [(schemes.SQUARE4_2_4, 4), (schemes.ORDER8_K6, 8)],
                         ids=["square4", "order8"])
def test_convergence_order_time_dependent(sch, order):
    # y' = w cos(w t) y, y(0) = 1, exact y = exp(sin(w t)), to T = 2, w = 4.
    # A wrong substep time t_n would cap the observed order at 1 or 2; the
    # extrapolated schemes approach their order from above (large
    # higher-order terms), hence the asymmetric window.
    steps, c = _cf(sch)
    w = 4.0
    f = lambda t, y: w * np.cos(w * t) * y
    errs = []
    for H in (1.0 / 8, 1.0 / 16):
        y = G.integrate(f, 0.0, np.array([1.0]), H, int(round(2.0 / H)), steps, c)
        errs.append(abs(y[0] - np.exp(np.sin(w * 2.0))))
    rate = np.log2(errs[0] / errs[1])
    assert order - 0.5 < rate < order + 1.5, (errs, rate)


def test_convergence_order_nonlinear():
    # pendulum q'' = -sin q as a first-order system; reference from a much
    # finer run of the same order-8 scheme
    steps, c = _cf(schemes.ORDER8_K6)
    f = lambda t, y: np.array([y[1], -np.sin(y[0])])
    y0 = np.array([1.0, 0.0])
    ref = G.integrate(f, 0.0, y0, 1.0 / 32, 128, steps, c)
    e = [np.max(np.abs(G.integrate(f, 0.0, y0, H, int(4 / H), steps, c) - ref))
         for H in (0.5, 0.25)]
    assert 7.5 < np.log2(e[0] / e[1]) < 9.5, e


def test_advection_direct_matches_spectral():
    cfg = workloads.CONFIG_ADVECTION1D
    steps, c = _cf(cfg["scheme"])
    u0 = fields.advection_modes(cfg["m"])
    op = OP.Advection1D(cfg["m"], r=2)
    direct = G.integrate(op, 0.0, u0, cfg["H"], cfg["n_macro"], steps, c)
    closed = SP.advection1d(u0, cfg["H"], steps, c, cfg["n_macro"])
    assert np.max(np.abs(direct - closed)) <= 1e-13 * np.max(np.abs(closed))


def test_acoustic_direct_matches_spectral():
    n = 64
    steps, c = _cf(schemes.ORDER8_K6)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / n, 2, workloads.SIGMA_FD4)
    y0 = fields.acoustic2d_pulse_modes(n, width=0.05)
    op = OP.Acoustic((n, n), c2=1.0, r=2)
    direct = G.integrate(op, 0.0, y0, H, 10, steps, c)
    closed = SP.acoustic(y0, 1.0, H, steps, c, 10)
    for k in range(3):
        assert np.max(np.abs(direct[k] - closed[k])) <= 1e-12 * np.max(np.abs(closed[0]))


@pytest.mark.parametrize("d", [2, 3])
def test_spectral_matches_dense_matrix_power(d):
    # brute force: build A column by column, evaluate sum_j c_j P_j(h_j A)
    # as a matrix polynomial and raise it to the n-th power
    shape = (6, 8) if d == 2 else (4, 4, 6)
    r = 2 if d == 2 else 4
    steps, c = _cf(schemes.ORDER8_K6)
    c2 = 1.7
    op = OP.Acoustic(shape, c2=c2, r=r)
    nstate = (1 + d) * int(np.prod(shape))
    a = np.zeros((nstate, nstate))
    for i in range(nstate):
        e = np.zeros(nstate)
        e[i] = 1.0
        a[:, i] = op.linear(e.reshape((1 + d,) + shape)).reshape(-1)
    H = 0.05
    rm = np.zeros_like(a)
    for n, ci in zip(steps, c):
        h = H / n
        coeffs = [q * Fraction(n) ** k for k, q in enumerate(S.gbs_poly(n))]
        acc = np.zeros_like(a)
        for q in reversed(coeffs):
            acc = acc @ (h * a) + float(q) * np.eye(nstate)
        rm += ci * acc
    nsteps = 7
    y0 = np.random.default_rng(5).standard_normal((1 + d,) + shape)
    want = (np.linalg.matrix_power(rm, nsteps) @ y0.reshape(-1)).reshape(y0.shape)
    got = SP.acoustic(y0, c2, H, steps, c, nsteps, r=r)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_converges_to_semidiscrete_solution():
    # against exp(t A) (the exact solution of the semi-discrete system):
    # halving H divides the error by 2^p
    m = 256
    u0 = fields.advection_modes(m)
    steps, c = _cf(schemes.SQUARE4_2_4)
    lam = -1j * SP.symbol(m, 1.0 / m, 2)
    exact = np.real(np.fft.ifft(np.fft.fft(u0) * np.exp(lam * 1.0)))
    errs = []
    for n in (131, 262):
        u = SP.advection1d(u0, 1.0 / n, steps, c, n)
        errs.append(np.max(np.abs(u - exact)))
    assert abs(np.log2(errs[0] / errs[1]) - 4) < 0.2, errs


def test_energy_non_increasing_variable_speed():
    # A is skew-adjoint in the inner product p^T C^{-2} p + |v|^2 and |R| <= 1
    # on the covered part of the imaginary axis, so that energy cannot grow
    n = 32
    cspeed = fields.lognormal_speed((n, n), seed=4)
    c2 = cspeed ** 2
    steps, c = _cf(schemes.ORDER8_K6)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cspeed.max(), 1.0 / n, 2,
                           workloads.SIGMA_FD4)
    op = OP.Acoustic((n, n), c2=c2, r=2)
    y = fields.acoustic2d_pulse_modes(n, width=0.08, seed=2)
    en = lambda y: 0.5 * (np.sum(y[0] ** 2 / c2) + np.sum(y[1:] ** 2))
    e_prev = en(y)
    for _ in range(20):
        y = G.macro_step(op, 0.0, y, H, steps, c)
        e = en(y)
        assert e <= e_prev * (1 + 1e-13)
        e_prev = e


def test_unstable_step_grows():
    # 1.3x the limit: energy must blow up eventually (the limit is sharp)
    n = 32
    steps, c = _cf(schemes.ORDER8_K6)
    H = 1.3 * workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / n, 2,
                                 workloads.SIGMA_FD4, frac=1.0)
    op = OP.Acoustic((n, n), c2=1.0, r=2)
    y = np.random.default_rng(0).standard_normal((3, n, n))
    y1 = G.integrate(op, 0.0, y, H, 40, steps, c)
    assert np.sum(y1 ** 2) > 1e3 * np.sum(y ** 2)


def test_periodic_window_reproduces_the_full_grid_at_its_centre():
    # the output of one macro step at a point depends on the input within
    # (N_max + 1) r points of it (each of the longest sequence's N_max + 1
    # evaluations reaches r points further), so the oracle run on a
    # periodic window of half-width W around a point, with the full grid's
    # spacing, gives the full grid's values at the window's centre points
    # within W - (N_max + 1) r of the middle: the same arithmetic, bitwise.
    # (2-D FD8 here; the 3-D full-size parity test samples its outputs so.)
    n, r, hw = 128, 4, 56
    steps, c = _cf(schemes.ORDER8_K6)
    reach = (max(steps) + 1) * r                        # 52
    cs = fields.lognormal_speed((n, n), seed=90)
    rng = np.random.default_rng(91)
    y0 = rng.standard_normal((3, n, n))
    H = 0.5 / n
    src_pt = (70, 40)
    ops = OP.Acoustic((n, n), c2=cs ** 2, r=r, sources=[OP.Source(src_pt, 9.0, 0.1, 50.0)])
    full = G.macro_step(ops, 0.09, y0, H, steps, c)
    ctr = (64, 37)
    iy, ix = [np.arange(q - hw, q + hw + 1) % n for q in ctr]
    win = np.ix_(iy, ix)
    local = tuple(p - (q - hw) for p, q in zip(src_pt, ctr))
    opw = OP.Acoustic((2 * hw + 1,) * 2, c2=(cs ** 2)[win], r=r, spacing=(1.0 / n, 1.0 / n),
                      sources=[OP.Source(local, 9.0, 0.1, 50.0)])
    part = G.macro_step(opw, 0.09, y0[(slice(None),) + win], H, steps, c)
    k = hw - reach                                       # exact half-width: 4
    inner = (slice(None), slice(hw - k, hw + k + 1), slice(hw - k, hw + k + 1))
    want = full[(slice(None),) + np.ix_(iy[hw - k:hw + k + 1], ix[hw - k:hw + k + 1])]
    assert np.array_equal(part[inner], want)
    # while near the window's edge its wrap has changed the values
    edge = full[(slice(None),) + np.ix_(iy[:8], ix)]
    assert np.abs(part[:, :8, :] - edge).max() > 1e-3 * np.abs(edge).max()
