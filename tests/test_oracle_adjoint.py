"""Pins for oracle.adjoint: the dot-product identity against the forward
oracle, and central finite differences of the misfit (exact for the initial
state since L is quadratic in it)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import adjoint as AD
from oracle import gbs as G
from oracle import operators as OP
from oracle import weights as W
from synth import fields, schemes, workloads


def _setup(n=16, with_source=True):
    sch = schemes.ORDER8_K6
    c = W.to_fp64(W.weights(8, sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]]))
    cs = fields.lognormal_speed((n, n), seed=11)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / n, 2, workloads.SIGMA_FD4)
    srcs = []
    if with_source:
        s = fields.ricker_source_2d(n, cells_per_wavelength=6.0)
        srcs = [OP.Source(s["idx"], s["f0"], s["delay"], s["weight"] * 1e-3)]
    op = OP.Acoustic((n, n), c2=c2, r=2, sources=srcs)
    return op, list(sch["steps"]), c, H


def test_dot_product_identity():
    op, steps, c, H = _setup(with_source=False)
    rng = np.random.default_rng(0)
    d = rng.standard_normal((3,) + op.shape)
    w = rng.standard_normal((3,) + op.shape)
    fwd = G.macro_step(op, 0.0, d, H, steps, c)
    adj, _ = AD.macro_step_adjoint(op, 0.0, np.zeros_like(d), H, steps, c, w, want_c2=False)
    assert np.sum(fwd * w) == pytest.approx(np.sum(d * adj), rel=1e-13)


def _problem(n_macro=3):
    op, steps, c, H = _setup()
    n = op.shape[0]
    rec = fields.edge_receivers_2d(n, count=8, row=2)
    y0 = fields.acoustic2d_pulse_modes(n, n_modes=4, kmax=3, width=0.1, seed=7)
    # synthetic data: a run with a perturbed coefficient
    c2_obs = op.c2 * np.exp(0.1 * fields.gaussian_random_field(op.shape, seed=12))
    op_obs = OP.Acoustic(op.shape, c2=c2_obs, r=2, sources=op.sources)
    _, ys = AD.misfit(op_obs, 0.0, y0, H, steps, c, n_macro, rec, np.zeros((n_macro, len(rec))))
    data = np.array([ys[k][0][rec[:, 0], rec[:, 1]] for k in range(1, n_macro + 1)])
    return op, steps, c, H, rec, y0, data, n_macro


def test_gradient_initial_state_vs_central_difference():
    op, steps, c, H, rec, y0, data, nm = _problem()
    L, gy, _ = AD.misfit_gradient(op, 0.0, y0, H, steps, c, nm, rec, data)
    rng = np.random.default_rng(3)
    for _ in range(3):
        d = rng.standard_normal(y0.shape)
        eps = 1e-3
        lp, _ = AD.misfit(op, 0.0, y0 + eps * d, H, steps, c, nm, rec, data)
        lm, _ = AD.misfit(op, 0.0, y0 - eps * d, H, steps, c, nm, rec, data)
        assert (lp - lm) / (2 * eps) == pytest.approx(np.sum(gy * d), rel=1e-8, abs=1e-12 * L)


def test_gradient_c2_vs_central_difference():
    op, steps, c, H, rec, y0, data, nm = _problem()
    L, _, gc = AD.misfit_gradient(op, 0.0, y0, H, steps, c, nm, rec, data)
    base = op.c2.copy()
    for seed in range(3):
        d = fields.gaussian_random_field(op.shape, ell=0.2, seed=100 + seed) * base
        eps = 1e-4
        vals = []
        for s in (+1, -1):
            op.c2 = base + s * eps * d
            vals.append(AD.misfit(op, 0.0, y0, H, steps, c, nm, rec, data)[0])
        op.c2 = base
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert fd == pytest.approx(np.sum(gc * d), rel=1e-6)


def _problem3d(n_macro=2):
    # 3-D FD8, two right-hand sides (each its own source) sharing c^2,
    # receivers on a z plane (index arrays (iz, iy, ix))
    shape = (8, 10, 12)
    sch = schemes.ORDER8_K6
    c = W.to_fp64(W.weights(8, sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]]))
    cs = fields.lognormal_speed(shape, seed=13)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / 12, 3, workloads.SIGMA_FD8)
    pts = [(2, 3, 4), (5, 7, 9)]
    f0, delay = 8.0, 0.05
    ops = [OP.Acoustic(shape, c2=c2, r=4, sources=[OP.Source(p, f0, delay, 50.0)]) for p in pts]
    recs = [np.array([[1, y, x] for y in (2, 6) for x in (1, 5, 10)]),
            np.array([[6, y, x] for y in (0, 4, 8) for x in (3, 7)])]
    rng = np.random.default_rng(14)
    y0s = [0.1 * rng.standard_normal((4,) + shape) for _ in pts]
    data = [0.05 * rng.standard_normal((n_macro, len(r))) for r in recs]
    return ops, list(sch["steps"]), c, H, y0s, recs, data, n_macro


def test_gradient_3d_two_rhs_initial_state_vs_central_difference():
    ops, steps, c, H, y0s, recs, data, nm = _problem3d()
    L, gys, _ = AD.misfit_gradient_rhs(ops, 0.01, y0s, H, steps, c, nm, recs, data)
    rng = np.random.default_rng(15)
    for r in range(2):
        d = rng.standard_normal(y0s[r].shape)
        eps = 1e-3
        vals = []
        for s in (1.0, -1.0):
            ys = [y.copy() for y in y0s]
            ys[r] = ys[r] + s * eps * d
            vals.append(AD.misfit_gradient_rhs(ops, 0.01, ys, H, steps, c, nm, recs, data)[0])
        # L is quadratic in y0: the central difference is exact up to rounding
        assert (vals[0] - vals[1]) / (2 * eps) == pytest.approx(np.sum(gys[r] * d), rel=1e-9)


def test_gradient_3d_two_rhs_c2_vs_central_difference():
    ops, steps, c, H, y0s, recs, data, nm = _problem3d()
    L, _, gc = AD.misfit_gradient_rhs(ops, 0.01, y0s, H, steps, c, nm, recs, data)
    base = ops[0].c2.copy()
    for seed in range(2):
        d = fields.gaussian_random_field(base.shape, ell=0.2, seed=200 + seed) * base
        eps = 1e-4
        vals = []
        for s in (1.0, -1.0):
            for op in ops:
                op.c2 = base + s * eps * d
            vals.append(AD.misfit_gradient_rhs(ops, 0.01, y0s, H, steps, c, nm, recs, data)[0])
        for op in ops:
            op.c2 = base
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert fd == pytest.approx(np.sum(gc * d), rel=1e-6)


def test_gradient_3d_receiver_index_order():
    # the receivers index the pressure field as (iz, iy, ix): the misfit of a
    # state that is zero except one pressure value equals 1/2 value^2 only at
    # the receiver whose index is that point
    ops, steps, c, H, y0s, recs, data, nm = _problem3d(n_macro=1)
    y = np.zeros((4,) + ops[0].shape)
    y[0][tuple(recs[0][2])] = 3.0
    at = AD._at(recs[0])
    vals = y[0][at]
    assert vals[2] == 3.0 and np.count_nonzero(vals) == 1
