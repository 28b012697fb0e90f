"""The RK4 comparison method on the library's stencil code against the
oracle's RK4 (1-D advection, 2-D acoustic with a c^2 field and a source,
3-D FD8 with two right-hand sides), and FP32 stepping against FP64."""
import math

import numpy as np
import pytest
import torch

from oracle import operators as OP
from oracle import rk4 as RK
from paper_1907_11771_amd import binding as B
from synth import fields, schemes, workloads
from tests.gpu_util import lib_plan, rel_err, to_dev

pytestmark = pytest.mark.gpu
RK4_ISB = 2 * math.sqrt(2)


def test_rk4_advection1d_vs_oracle():
    m = 256
    u0 = fields.advection_modes(m, seed=0)
    h = 0.8 * RK4_ISB / (workloads.SIGMA_FD4 * m)
    plan = lib_plan(B.ADVECT1D, (m,), schemes.SQUARE4_2_4, h)
    got = plan.rk4_step(to_dev(u0[None]), n_steps=40).cpu().numpy()[0]
    want = RK.integrate(OP.Advection1D(m, r=2), 0.0, u0, h, 40)
    assert rel_err(got, want, 0) <= 1e-12


def test_rk4_acoustic2d_c2_field_source_in_place_vs_oracle():
    ny, nx = 72, 90
    cs = fields.lognormal_speed((ny, nx), seed=80)
    c2 = cs ** 2
    h = workloads.stable_H(RK4_ISB, cs.max(), 1.0 / nx, 2, workloads.SIGMA_FD4)
    s = fields.ricker_source_2d(nx, cells_per_wavelength=8.0)
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), schemes.ORDER8_K6, 1e-6, c2_field=to_dev(c2),
                    c_max=float(cs.max()))
    plan.set_sources([0], [30 * nx + 41], [s["weight"] * 1e-3], s["f0"], s["delay"])
    y0 = np.random.default_rng(81).standard_normal((3, ny, nx))
    t0 = s["delay"] - 5 * h
    y = to_dev(y0[None])
    plan.rk4_step(y, y, t0=t0, n_steps=12, h=h)
    op = OP.Acoustic((ny, nx), c2=c2, r=2,
                     sources=[OP.Source((30, 41), s["f0"], s["delay"], s["weight"] * 1e-3)])
    want = RK.integrate(op, t0, y0, h, 12)
    assert rel_err(y.cpu().numpy()[0], want, 0) <= 1e-12


def test_rk4_acoustic3d_fd8_two_rhs_vs_oracle():
    shape = (14, 12, 18)
    cs = fields.lognormal_speed(shape, seed=82)
    c2 = cs ** 2
    h = workloads.stable_H(RK4_ISB, cs.max(), 1.0 / 18, 3, workloads.SIGMA_FD8)
    plan = lib_plan(B.ACOUSTIC3D, (18, 12, 14), schemes.ORDER8_K6, 1e-6, fd_order=8, n_rhs=2,
                    c2_field=to_dev(c2), c_max=float(cs.max()))
    y0 = np.random.default_rng(83).standard_normal((2, 4) + shape)
    got = plan.rk4_step(to_dev(y0), n_steps=6, h=h).cpu().numpy()
    op = OP.Acoustic(shape, c2=c2, r=4)
    for r in range(2):
        assert rel_err(got[r], RK.integrate(op, 0.0, y0[r], h, 6), 0) <= 1e-12


def test_rk4_fp32_stepping_error_and_stability_check():
    n = 128
    h = workloads.stable_H(RK4_ISB, 1.0, 1.0 / n, 2, workloads.SIGMA_FD4)
    y0 = fields.acoustic2d_pulse_modes(n, n_modes=8, kmax=6, width=0.05, seed=4)
    p64 = lib_plan(B.ACOUSTIC2D, (n, n), schemes.ORDER8_K6, 1e-6)
    p32 = lib_plan(B.ACOUSTIC2D, (n, n), schemes.ORDER8_K6, 1e-6, dtype=torch.float32)
    a = p64.rk4_step(to_dev(y0[None]), n_steps=50, h=h).cpu().numpy()
    b = p32.rk4_step(to_dev(y0[None], torch.float32), n_steps=50, h=h).cpu().numpy()
    err = rel_err(b, a, 1)
    print("rk4 fp32 vs fp64", err)
    assert err <= 2e-5
    with pytest.raises(B.GBSError) as ei:
        p64.rk4_step(to_dev(y0[None]), n_steps=1, h=1.01 * h / 0.8)
    assert ei.value.status == B.GBS_EUNSTABLE


def test_fine_run_reference_of_the_time_to_solution_comparison():
    # the comparison measures errors against the same scheme at H/4; here
    # that estimate is checked against the semi-discrete solution exp(tA) y0
    from oracle import spectral as SP
    from paper_1907_11771_amd.plan import scheme_weights
    n, nm = 128, 20
    steps, w, isb = scheme_weights(schemes.ORDER8_K6)
    H = workloads.stable_H(isb, 1.0, 1.0 / n, 2, workloads.SIGMA_FD4)
    y0 = fields.acoustic2d_pulse_modes(n, n_modes=8, kmax=6, width=0.1, seed=5)
    exact = SP.acoustic_exact(y0, 1.0, nm * H)
    coarse = lib_plan(B.ACOUSTIC2D, (n, n), schemes.ORDER8_K6, H)
    fine = lib_plan(B.ACOUSTIC2D, (n, n), schemes.ORDER8_K6, H / 4)
    yc = coarse.step(to_dev(y0[None]), n_macro=nm).cpu().numpy()[0]
    yf = fine.step(to_dev(y0[None]), n_macro=4 * nm).cpu().numpy()[0]
    e_true = np.max(np.abs(yc - exact))
    e_fine = np.max(np.abs(yf - exact))
    e_est = np.max(np.abs(yc - yf))
    print("coarse", e_true, "fine", e_fine, "estimate", e_est)
    assert e_fine <= e_true / 1000
    assert abs(e_est - e_true) <= 0.01 * e_true
