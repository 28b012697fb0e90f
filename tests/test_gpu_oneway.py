"""The paper's experiment (Sect. 4.1) through the library: the one-way wave
equation with the Fourier derivative (fd_order = GBS_FD_SPECTRAL), one
revolution at 0.99 of each method's limit, GBS_{8,6}, GBS_{12,8} and RK4,
against the oracle's literal FP64 runs and the extended-precision fully
discrete solution; even and odd M; several right-hand sides; FP32 stepping."""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import oneway as O
from oracle import stability as S
from oracle import weights as W
from paper_1907_11771_amd import binding as B
from paper_1907_11771_amd.plan import GBSPlan, scheme_weights
from synth import schemes
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu
RK4_ISB = 2 * math.sqrt(2)


def _plan(sch, m, n, n_rhs=1, dtype=torch.float64):
    steps, w, _ = scheme_weights(sch)
    return GBSPlan(B.ADVECT1D, (m,), sch["p"], steps, w, 1.0 / n, fd_order=B.FD_SPECTRAL,
                   n_rhs=n_rhs, dtype=dtype), steps, w


def _isb(sch):
    c = W.weights(sch["p"], list(sch["steps"]), sch["free_idx"],
                  [Fraction(x) for x in sch["c_free"]])
    return float(S.isb(S.extrapolated_poly(list(sch["steps"]), c)))


@pytest.mark.parametrize("sch,ms", [(schemes.GBS_8_6, (16, 33, 64)), (schemes.GBS_12_8, (16, 33))],
                         ids=["gbs_8_6", "gbs_12_8"])
def test_one_revolution_vs_oracle(sch, ms):
    for m in ms:
        n, _ = O.macro_steps(m, _isb(sch))
        plan, steps, w = _plan(sch, m, n)
        got = plan.step(to_dev(O.initial(m)[None]), n_macro=n).cpu().numpy()[0]
        want, e_want = O.run(m, steps, w, n)
        d = float(np.max(np.abs(got - want)))
        print(sch["name"], "M", m, "n", n, "|gpu - oracle|", d, "error", e_want)
        assert d <= 1e-12, (m, d)


@pytest.mark.parametrize("sch", [schemes.GBS_8_6, schemes.GBS_12_8], ids=["gbs_8_6", "gbs_12_8"])
def test_as_close_to_the_fully_discrete_solution_as_the_oracle(sch):
    # at the FP64 floor both runs differ from the exact fully discrete
    # solution by their own rounding; the library may not be worse than
    # the oracle by more than a small factor
    for m in (64, 128):
        n, _ = O.macro_steps(m, _isb(sch))
        plan, steps, w = _plan(sch, m, n)
        exact = O.solution_closed_form(m, O.gbs_poly(steps, w), n)
        got = plan.step(to_dev(O.initial(m)[None]), n_macro=n).cpu().numpy()[0]
        lit, _ = O.run(m, steps, w, n)
        d_gpu = float(np.max(np.abs(got - exact)))
        d_or = float(np.max(np.abs(lit - exact)))
        print(sch["name"], "M", m, "gpu", d_gpu, "oracle", d_or)
        assert d_gpu <= 4 * d_or + 1e-15, (m, d_gpu, d_or)


def test_rk4_one_revolution_vs_oracle():
    for m in (16, 33):
        n, _ = O.macro_steps(m, RK4_ISB)
        plan, _, _ = _plan(schemes.GBS_8_6, m, 4 * m)         # any scheme: RK4 uses the operator
        got = plan.rk4_step(to_dev(O.initial(m)[None]), n_steps=n, h=1.0 / n).cpu().numpy()[0]
        want, e_want = O.run_rk4(m, n)
        print("rk4 M", m, "n", n, "|gpu - oracle|", float(np.max(np.abs(got - want))), e_want)
        assert np.max(np.abs(got - want)) <= 1e-12


def test_right_hand_sides_are_independent():
    m, sch = 40, schemes.GBS_8_6
    n, _ = O.macro_steps(m, _isb(sch))
    plan, steps, w = _plan(sch, m, n, n_rhs=3)
    rng = np.random.default_rng(90)
    y0 = rng.standard_normal((3, 1, m))
    got = plan.step(to_dev(y0), n_macro=3).cpu().numpy()
    one, _, _ = _plan(sch, m, n)
    from oracle import gbs as G
    from oracle import operators as OP
    for r in range(3):
        single = one.step(to_dev(y0[r:r + 1]), n_macro=3).cpu().numpy()[0]
        assert np.array_equal(single, got[r])
        want = G.integrate(OP.SpectralAdvection1D(m), 0.0, y0[r], 1.0 / n, 3, steps, w)
        assert np.max(np.abs(got[r] - want)) <= 1e-12 * np.max(np.abs(want))


def test_fp32_stepping():
    m, sch = 64, schemes.GBS_8_6
    n, _ = O.macro_steps(m, _isb(sch))
    p64, _, _ = _plan(sch, m, n)
    p32, _, _ = _plan(sch, m, n, dtype=torch.float32)
    u0 = O.initial(m)[None]
    a = p64.step(to_dev(u0), n_macro=n).cpu().numpy()
    b = p32.step(to_dev(u0, torch.float32), n_macro=n).cpu().numpy()
    err = float(np.max(np.abs(a - b)))
    print("fp32 vs fp64 after one revolution", err)
    # FP32 levels: rounding 6e-8 per level, amplified by sum |c| = 31
    assert err <= 1e-5


@pytest.mark.parametrize("m,n_macro", [(4, 3), (5, 3), (8192, 2)])
def test_smallest_and_largest_grids(m, n_macro):
    # 4 and 5 points: one weight b_1 (K = 1, resp. 2); 8192: the largest grid
    # the Fourier derivative accepts; random data, a few macro steps
    sch = schemes.GBS_8_6
    n, _ = O.macro_steps(m, _isb(sch))
    plan, steps, w = _plan(sch, m, n)
    y0 = np.random.default_rng(m).standard_normal((1, m))
    got = plan.step(to_dev(y0[None]), n_macro=n_macro).cpu().numpy()[0]
    from oracle import gbs as G
    from oracle import operators as OP
    want = G.integrate(OP.SpectralAdvection1D(m), 0.0, y0, 1.0 / n, n_macro, steps, w)
    err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    print("M", m, "rel err", err)
    assert err <= 1e-12
