"""gbs_step_scratch (the entry point that allocates nothing: its workspace is
the library's static device array) against gbs_step on a plan with its own
workspace, through the C ABI: two calls in a row, the second on a smaller
problem, must give the same states; a problem beyond the array's size is
refused."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1907_11771_amd import binding as B
from paper_1907_11771_amd.plan import scheme_weights
from synth import fields, schemes, workloads
from tests.gpu_util import lib_plan, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _scratch_step(op, n, sch, H, y, t0, n_macro, dtype=torch.float64, **kw):
    steps, w, _ = scheme_weights(sch)
    prob = B.make_problem(op, n, kw.get("fd_order", 4), y.shape[0],
                          B.F64 if dtype == torch.float64 else B.F32, 1.0, None, 0.0,
                          kw.get("flags", 0))
    scheme = B.make_scheme(sch["p"], steps, w)
    out = torch.empty_like(y)
    B.check(B.lib().gbs_step_scratch(ctypes.byref(prob), ctypes.byref(scheme), float(H),
                                     float(t0), int(n_macro), y.data_ptr(), out.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream))
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_scratch_step_equals_plan_step_twice_then_smaller(dtype):
    sch = schemes.ORDER8_K6
    # first call: 2-D acoustic 120 x 96, two right-hand sides; second: 64 x 40
    for (nx, ny), nrhs, seed in (((120, 96), 2, 1), ((64, 40), 1, 2)):
        H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / max(nx, ny), 2,
                               workloads.SIGMA_FD4)
        y0 = to_dev(np.random.default_rng(seed).standard_normal((nrhs, 3, ny, nx)), dtype)
        plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, n_rhs=nrhs, dtype=dtype)
        want = plan.step(y0, t0=0.25, n_macro=3)
        got = _scratch_step(B.ACOUSTIC2D, (nx, ny), sch, H, y0, 0.25, 3, dtype)
        torch.cuda.synchronize()
        assert torch.equal(got, want), rel_err(got.double().cpu().numpy(),
                                               want.double().cpu().numpy(), 1)


def test_scratch_step_3d_and_1d():
    sch = schemes.ORDER8_K6
    shape = (12, 20, 24)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / 24, 3, workloads.SIGMA_FD8)
    y0 = to_dev(np.random.default_rng(3).standard_normal((2, 4) + shape))
    plan = lib_plan(B.ACOUSTIC3D, (24, 20, 12), sch, H, fd_order=8, n_rhs=2)
    want = plan.step(y0, n_macro=2)
    got = _scratch_step(B.ACOUSTIC3D, (24, 20, 12), sch, H, y0, 0.0, 2, fd_order=8)
    assert torch.equal(got, want)
    cfg = workloads.CONFIG_ADVECTION1D
    u0 = to_dev(fields.advection_modes(cfg["m"]).reshape(1, 1, -1))
    plan = lib_plan(B.ADVECT1D, (cfg["m"],), cfg["scheme"], cfg["H"])
    want = plan.step(u0, n_macro=7)
    got = _scratch_step(B.ADVECT1D, (cfg["m"],), cfg["scheme"], cfg["H"], u0, 0.0, 7)
    assert torch.equal(got, want)


def test_scratch_step_refuses_a_problem_beyond_the_array():
    sch = schemes.ORDER8_K6
    n = 1024                       # 1024^2 FP64 needs far more than the array holds
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / n, 2, workloads.SIGMA_FD4)
    y = torch.zeros((1, 3, n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(B.GBSError) as ei:
        _scratch_step(B.ACOUSTIC2D, (n, n), sch, H, y, 0.0, 1)
    assert ei.value.status == B.GBS_ENOMEM
    assert "scratch" in str(ei.value)
