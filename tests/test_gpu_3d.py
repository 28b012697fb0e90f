"""The 3-D FD8 multi-right-hand-side workload at the parity grid (96^3, the
384^3 field sampled every 4th point, the same 8 source positions): FP64
against the oracle, FP32 stepping against the oracle with a stated bound,
the right-hand sides of one batched plan against single-source plans, and
the adjoint against the oracle's discrete adjoint."""
import numpy as np
import pytest
import torch

from oracle import adjoint as AD
from oracle import gbs as G
from oracle import operators as OP
from paper_1907_11771_amd import binding as B
from synth import fields, schemes, workloads
from tests.gpu_util import lib_plan, oracle_weights, rel_err, to_dev

pytestmark = pytest.mark.gpu

N = 96
TOL64 = 1e-12
# FP32 levels with the FP64 averaging and combination, one macro step from
# unit-variance data: measured ~1e-6; bound u32 * sum|c| * (1 + sum N_j)
# rounded up (6e-8 * 12 * 43 = 3e-5)
TOL32 = 3e-5


def _setup():
    cs = fields.bandlimited_lognormal_speed(N, seed=workloads.CONFIG_3D["speed_seed"],
                                            kmax=workloads.CONFIG_3D["kmax"])
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / N, 3, workloads.SIGMA_FD8)
    src = fields.ricker_source_3d(N, workloads.sources_3d(N, seed=workloads.CONFIG_3D["source_seed"]))
    return cs ** 2, float(cs.max()), H, src


def _plan(c2, cmax, H, src, rhs_sources, dtype):
    plan = lib_plan(B.ACOUSTIC3D, (N, N, N), schemes.ORDER8_K6, H, fd_order=8,
                    n_rhs=len(rhs_sources), dtype=dtype, c2_field=to_dev(c2, dtype), c_max=cmax)
    flat = [z * N * N + y * N + x for z, y, x in (src["points"][i] for i in rhs_sources)]
    plan.set_sources(list(range(len(rhs_sources))), flat, [src["weight"]] * len(rhs_sources),
                     src["f0"], src["delay"])
    return plan


def test_acoustic3d_96_eight_sources_fp64_fp32_vs_oracle():
    c2, cmax, H, src = _setup()
    steps, c = oracle_weights(schemes.ORDER8_K6)
    rng = np.random.default_rng(60)
    y0 = rng.standard_normal((8, 4, N, N, N))
    t0 = src["delay"] - 0.5 * H               # the source near its peak
    out = {}
    for dtype in (torch.float64, torch.float32):
        plan = _plan(c2, cmax, H, src, range(8), dtype)
        out[dtype] = plan.step(to_dev(y0, dtype), t0=t0, n_macro=1).double().cpu().numpy()
    # the oracle for two of the right-hand sides (7.5 s each on one core)
    for r in (0, 5):
        op = OP.Acoustic((N, N, N), c2=c2, r=4,
                         sources=[OP.Source(src["points"][r], src["f0"], src["delay"],
                                            src["weight"])])
        want = G.macro_step(op, t0, y0[r], H, steps, c)
        e64 = rel_err(out[torch.float64][r], want)
        e32 = rel_err(out[torch.float32][r], want)
        print("rhs", r, "fp64 vs oracle", e64, "fp32 vs oracle", e32)
        assert e64 <= TOL64
        assert e32 <= TOL32
    # every right-hand side of the batched plan equals a plan with that
    # source alone (the right-hand sides share only c^2)
    for r in (1, 2, 3, 4, 6, 7):
        single = _plan(c2, cmax, H, src, [r], torch.float64)
        got = single.step(to_dev(y0[r:r + 1]), t0=t0, n_macro=1).cpu().numpy()[0]
        assert np.array_equal(got, out[torch.float64][r]), r


def test_acoustic3d_96_adjoint_vs_oracle_and_fp32():
    c2, cmax, H, src = _setup()
    steps, c = oracle_weights(schemes.ORDER8_K6)
    rng = np.random.default_rng(61)
    y0 = rng.standard_normal((1, 4, N, N, N))
    wbar = rng.standard_normal((1, 4, N, N, N))
    t0 = src["delay"] - 0.5 * H               # the source (it enters the c^2 gradient) near its peak
    res = {}
    for dtype in (torch.float64, torch.float32):
        plan = _plan(c2, cmax, H, src, [0], dtype)
        ybar = to_dev(wbar, dtype)
        grad = torch.zeros((N, N, N), dtype=torch.float64, device="cuda")
        plan.adjoint_step(t0, to_dev(y0, dtype), ybar, grad_c2=grad)
        res[dtype] = (ybar.double().cpu().numpy()[0], grad.cpu().numpy())
    op = OP.Acoustic((N, N, N), c2=c2, r=4,
                     sources=[OP.Source(src["points"][0], src["f0"], src["delay"], src["weight"])])
    want_y, want_g = AD.macro_step_adjoint(op, t0, y0[0], H, steps, c, wbar[0])
    assert rel_err(res[torch.float64][0], want_y) <= TOL64
    assert rel_err(res[torch.float64][1], want_g) <= TOL64
    e_y = rel_err(res[torch.float32][0], want_y)
    e_g = rel_err(res[torch.float32][1], want_g)
    print("fp32 adjoint vs oracle: ybar", e_y, "grad", e_g)
    assert e_y <= TOL32 and e_g <= TOL32
