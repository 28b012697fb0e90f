"""The paper's published schemes through the same kernels: the fully
determined optimum schemes of order 8, 12 and 16 (Sect. 3.3, Table 1) and
the methods of choice GBS_{8,6}, GBS_{8,8} and GBS_{12,8} (Sect. 3.8; up to
15 sequences, N_max = 30), and the smallest scheme, order 4 over N = {2, 4}
(two sequences, one blocked launch), each on a 2-D acoustic problem with a
c^2 field and a source at 0.8 of the scheme's own stability limit, in the
blocked and the streaming forms, against the oracle."""
import numpy as np
import pytest
import torch

from oracle import gbs as G
from oracle import operators as OP
from paper_1907_11771_amd import binding as B
from paper_1907_11771_amd.plan import scheme_weights
from synth import fields, schemes, workloads
from tests.gpu_util import lib_plan, oracle_weights, rel_err, to_dev

pytestmark = pytest.mark.gpu

PUBLISHED = [schemes.FULLDET8, schemes.FULLDET12, schemes.FULLDET16, schemes.GBS_8_6,
             schemes.GBS_8_8, schemes.GBS_12_8, schemes.SQUARE4_2_4]


@pytest.mark.parametrize("sch", PUBLISHED, ids=[s["name"] for s in PUBLISHED])
def test_published_scheme_vs_oracle(sch):
    ny, nx = 72, 80
    steps, c = oracle_weights(sch)
    _, _, isb = scheme_weights(sch)
    cs = fields.lognormal_speed((ny, nx), seed=70)
    c2 = cs ** 2
    H = workloads.stable_H(isb, cs.max(), 1.0 / nx, 2, workloads.SIGMA_FD4)
    s = fields.ricker_source_2d(nx, cells_per_wavelength=8.0)
    y0 = np.random.default_rng(71).standard_normal((3, ny, nx))
    t0 = s["delay"] - H
    op = OP.Acoustic((ny, nx), c2=c2, r=2,
                     sources=[OP.Source((30, 41), s["f0"], s["delay"], s["weight"] * 1e-3)])
    want = G.integrate(op, t0, y0, H, 2, steps, c)
    # the combination amplifies the levels' rounding by sum |c_j| (up to 582
    # for GBS_{12,8}); the tolerance stays 1e-12 relative
    for v in (B.VARIANT_AUTO, B.VARIANT_FLAT):
        plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, c2_field=to_dev(c2),
                        c_max=float(cs.max()))
        plan.set_sources([0], [30 * nx + 41], [s["weight"] * 1e-3], s["f0"], s["delay"])
        plan.set_variant(v)
        got = plan.step(to_dev(y0[None]), t0=t0, n_macro=2).cpu().numpy()[0]
        err = rel_err(got, want, 0)
        print(sch["name"], "variant", v, "rel err", err, "sum|c|", float(np.sum(np.abs(c))))
        assert err <= 1e-12, (sch["name"], v, err)
