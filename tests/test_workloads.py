"""The workload constants (stability-limit inputs) against the oracle."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import stability as S
from oracle import spectral as SP
from oracle import weights as W
from synth import fields, schemes, workloads


def _sup_symbol(r):
    # max over theta of s(theta) (dx = 1), dense grid then golden refinement
    th = np.linspace(0, np.pi, 200001)
    s = SP.symbol(2, 1.0, r)  # warm the cache of weights
    from oracle.operators import centred_first_derivative_weights
    a = [float(x) for x in centred_first_derivative_weights(r)]
    f = lambda t: sum(2 * ak * np.sin((k + 1) * t) for k, ak in enumerate(a))
    i = int(np.argmax(f(th)))
    lo, hi = th[max(i - 1, 0)], th[min(i + 1, len(th) - 1)]
    g = (np.sqrt(5) - 1) / 2
    for _ in range(100):
        m1, m2 = hi - g * (hi - lo), lo + g * (hi - lo)
        if f(m1) < f(m2):
            lo = m1
        else:
            hi = m2
    return f(0.5 * (lo + hi))


def test_sigma_constants_round_up():
    for r, lit in ((2, workloads.SIGMA_FD4), (4, workloads.SIGMA_FD8)):
        s = _sup_symbol(r)
        assert s <= lit < s + 2e-7


@pytest.mark.parametrize("sch,lit", [(schemes.ORDER8_K6, workloads.ISB_ORDER8_K6),
                                     (schemes.SQUARE4_2_4, workloads.ISB_SQUARE4)])
def test_isb_constants_round_down(sch, lit):
    c = W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    isb = S.isb(S.extrapolated_poly(sch["steps"], c))
    assert isb - 1e-3 < lit <= isb


def test_config_steps_are_within_the_limit():
    cfg = workloads.CONFIG_ADVECTION1D
    lim = workloads.stable_H(workloads.ISB_SQUARE4, 1.0, 1.0 / cfg["m"], 1, workloads.SIGMA_FD4, 1.0)
    assert 0.79 * lim < cfg["H"] <= 0.8 * lim
    assert cfg["H"] * cfg["n_macro"] == pytest.approx(1.0)
    cfg = workloads.CONFIG_ACOUSTIC2D
    lim = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / cfg["n"], 2, workloads.SIGMA_FD4, 1.0)
    assert cfg["H"] == pytest.approx(0.8 * lim, rel=1e-12)


def test_bandlimited_field_is_grid_independent():
    # the 96^3 parity grid samples the 384^3 workload's field every 4th point;
    # checked here at 24^3 against 48^3 (same property, smaller grids)
    a = fields.bandlimited_lognormal_speed(48, d=3, kmax=8, seed=50)
    b = fields.bandlimited_lognormal_speed(24 * 4, d=3, kmax=8, seed=50)
    assert np.abs(b[::2, ::2, ::2] - a).max() < 1e-12
    assert a.min() > 0
    g = np.log(a) / 0.2
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12


def test_3d_sources_sit_on_the_coarse_lattice():
    fine = workloads.sources_3d(384)
    coarse = workloads.sources_3d(96)
    assert len(set(fine)) == 8
    assert [tuple(4 * v for v in p) for p in coarse] == fine
