"""GPU parity: the HIP library against the CPU oracle on identical seeded
inputs.  FP64 bar: max |gpu - oracle| / max |oracle| <= 1e-12 per field."""
import numpy as np
import pytest
import torch

from oracle import gbs as G
from oracle import operators as OP
from oracle import spectral as SP
from paper_1907_11771_amd import binding as B
from synth import fields, schemes, workloads
from tests.gpu_util import lib_plan, oracle_weights, rel_err, to_dev

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def test_weights_used_by_plan_are_the_oracles():
    for sch in (schemes.SQUARE4_2_4, schemes.ORDER8_K6):
        plan = lib_plan(B.ADVECT1D, (64,), sch, 1e-4)
        assert plan.w == oracle_weights(sch)[1]


def test_advection1d_config_vs_oracle_and_closed_form():
    cfg = workloads.CONFIG_ADVECTION1D
    steps, c = oracle_weights(cfg["scheme"])
    u0 = fields.advection_modes(cfg["m"])
    plan = lib_plan(B.ADVECT1D, (cfg["m"],), cfg["scheme"], cfg["H"])
    y = to_dev(u0.reshape(1, 1, -1))
    out = plan.step(y, n_macro=cfg["n_macro"])
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(1, -1)
    direct = G.integrate(OP.Advection1D(cfg["m"]), 0.0, u0, cfg["H"], cfg["n_macro"], steps, c)
    closed = SP.advection1d(u0, cfg["H"], steps, c, cfg["n_macro"])
    assert rel_err(got, direct, 0) <= TOL64
    assert rel_err(got, closed, 0) <= TOL64


@pytest.mark.parametrize("shape,order", [((72, 100), 4), ((40, 56), 8), ((33, 17), 4)])
def test_acoustic2d_constant_c_vs_oracle(shape, order):
    ny, nx = shape
    sch = schemes.ORDER8_K6
    steps, c = oracle_weights(sch)
    sig = workloads.SIGMA_FD4 if order == 4 else workloads.SIGMA_FD8
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / max(nx, ny), 2, sig)
    rng = np.random.default_rng(7)
    y0 = rng.standard_normal((3, ny, nx))
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, fd_order=order, check_stability=False)
    out = plan.step(to_dev(y0[None]), n_macro=4)
    got = out.cpu().numpy()[0]
    want = G.integrate(OP.Acoustic((ny, nx), c2=1.0, r=order // 2), 0.0, y0, H, 4, steps, c)
    for q in range(3):
        assert rel_err(got[q], want[q], None) <= TOL64, q


def test_acoustic2d_variable_c2_with_source_vs_oracle():
    n = 96
    sch = schemes.ORDER8_K6
    steps, c = oracle_weights(sch)
    cs = fields.lognormal_speed((n, n), seed=21)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / n, 2, workloads.SIGMA_FD4)
    s = fields.ricker_source_2d(n, cells_per_wavelength=8.0)
    y0 = fields.acoustic2d_pulse_modes(n, n_modes=6, kmax=4, width=0.05, seed=3)
    plan = lib_plan(B.ACOUSTIC2D, (n, n), sch, H, c2_field=to_dev(c2), c_max=float(cs.max()))
    flat = s["idx"][0] * n + s["idx"][1]
    plan.set_sources([0], [flat], [s["weight"]], s["f0"], s["delay"])
    n_macro = 6
    t0 = 0.25 * s["delay"]
    out = plan.step(to_dev(y0[None]), t0=t0, n_macro=n_macro)
    got = out.cpu().numpy()[0]
    op = OP.Acoustic((n, n), c2=c2, r=2,
                     sources=[OP.Source(s["idx"], s["f0"], s["delay"], s["weight"])])
    want = G.integrate(op, t0, y0, H, n_macro, steps, c)
    for q in range(3):
        assert rel_err(got[q], want[q], None) <= TOL64, q


@pytest.mark.parametrize("variant", [B.VARIANT_AUTO, B.VARIANT_TILE3D])
def test_acoustic3d_fd8_variable_c2_multi_rhs_vs_oracle(variant):
    shape = (12, 20, 24)   # z, y, x
    sch = schemes.ORDER8_K6
    steps, c = oracle_weights(sch)
    cs = fields.lognormal_speed(shape, seed=5)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / 24, 3, workloads.SIGMA_FD8)
    rng = np.random.default_rng(9)
    y0 = rng.standard_normal((2, 4) + shape)
    plan = lib_plan(B.ACOUSTIC3D, (24, 20, 12), sch, H, fd_order=8, n_rhs=2,
                    c2_field=to_dev(c2), c_max=float(cs.max()))
    srcs = [(0, (6, 10, 12)), (1, (3, 4, 5))]
    flat = [z * 20 * 24 + y * 24 + x for _, (z, y, x) in srcs]
    f0, delay = 30.0, 0.05
    plan.set_sources([0, 1], flat, [50.0, -20.0], f0, delay)
    plan.set_variant(variant)
    out = plan.step(to_dev(y0), n_macro=3)
    got = out.cpu().numpy()
    for r, (w_, (idx)) in enumerate(zip([50.0, -20.0], [srcs[0][1], srcs[1][1]])):
        op = OP.Acoustic(shape, c2=c2, r=4, sources=[OP.Source(idx, f0, delay, w_)])
        want = G.integrate(op, 0.0, y0[r], H, 3, steps, c)
        for q in range(4):
            assert rel_err(got[r, q], want[q], None) <= TOL64, (r, q)


def test_in_place_and_repeatable():
    n = 64
    sch = schemes.ORDER8_K6
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / n, 2, workloads.SIGMA_FD4)
    y0 = to_dev(np.random.default_rng(1).standard_normal((1, 3, n, n)))
    plan = lib_plan(B.ACOUSTIC2D, (n, n), sch, H)
    a = plan.step(y0, n_macro=5)
    b = plan.step(y0, n_macro=5)
    c = y0.clone()
    plan.step(c, out=c, n_macro=5)
    assert torch.equal(a, b) and torch.equal(a, c)
    z = plan.step(y0, n_macro=0)
    assert torch.equal(z, y0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_kernel_variants_agree_bitwise(dtype):
    # every leap-frog variant computes the same values in the same order
    ny, nx = 200, 136                   # ragged in both directions
    sch = schemes.ORDER8_K6
    cs = fields.lognormal_speed((ny, nx), seed=2)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    y0 = to_dev(np.random.default_rng(3).standard_normal((2, 3, ny, nx)), dtype)
    outs = []
    for v in (B.VARIANT_FLAT, B.VARIANT_MARCH8, B.VARIANT_MARCH16, B.VARIANT_MARCH8_NT,
              B.VARIANT_MARCH16_NT, B.VARIANT_PLAIN):
        plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, n_rhs=2, dtype=dtype,
                        c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()))
        plan.set_variant(v)
        outs.append(plan.step(y0, n_macro=3))
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_3d_kernel_variants_agree_bitwise(dtype):
    # z-marching (64 and 128 planes per thread), flat and per-sequence forms
    shape = (70, 22, 90)                # z, y, x: ragged against 64 / 4 / 64
    sch = schemes.ORDER8_K6
    cs = fields.lognormal_speed(shape, seed=12)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / 90, 3, workloads.SIGMA_FD8)
    y0 = to_dev(np.random.default_rng(13).standard_normal((2, 4) + shape), dtype)
    outs = []
    for v in (B.VARIANT_FLAT, B.VARIANT_MARCH8, B.VARIANT_MARCH16, B.VARIANT_PLAIN):
        plan = lib_plan(B.ACOUSTIC3D, (90, 22, 70), sch, H, fd_order=8, n_rhs=2, dtype=dtype,
                        c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()))
        plan.set_sources([1], [(35 * 22 + 11) * 90 + 45], [1e3], 20.0, 0.01)
        plan.set_variant(v)
        outs.append(plan.step(y0, t0=0.005, n_macro=2))
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("variant,band", [(B.VARIANT_TEMPORAL, 128), (B.VARIANT_TEMPORAL, 7),
                                          (B.VARIANT_TEMPORAL4, 50), (B.VARIANT_TEMPORAL, 1000),
                                          (B.VARIANT_TEMPORAL_S5, 64), (B.VARIANT_TEMPORAL_S6, 33),
                                          (B.VARIANT_TEMPORAL_WG4, 64), (B.VARIANT_TEMPORAL_WG8, 20),
                                          (B.VARIANT_TEMPORAL_WG8, 128), (B.VARIANT_TEMPORAL_S5, 0),
                                          (B.VARIANT_TEMPORAL, 0)])
def test_temporal_passes_match_streaming(dtype, variant, band):
    # temporally blocked passes against the streaming sweeps: same values up
    # to the contraction of products (and FP32 rounding of the levels)
    ny, nx = 200, 136
    sch = schemes.ORDER8_K6
    cs = fields.lognormal_speed((ny, nx), seed=2)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    y0 = to_dev(np.random.default_rng(3).standard_normal((2, 3, ny, nx)), dtype)
    s = fields.ricker_source_2d(max(nx, ny), cells_per_wavelength=8.0)
    res = []
    for v in (B.VARIANT_FLAT, variant):
        plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, n_rhs=2, dtype=dtype,
                        c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()))
        plan.set_sources([1], [77 * nx + 50], [s["weight"] * 1e-4], s["f0"], s["delay"])
        plan.set_variant(v)
        if v != B.VARIANT_FLAT:
            B.check(B.lib().gbs_plan_set_band(plan.handle, band))
        res.append(plan.step(y0, t0=0.3 * s["delay"], n_macro=3).cpu().numpy())
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    assert rel_err(res[1], res[0], 1) <= tol


@pytest.mark.parametrize("variant", [B.VARIANT_TEMPORAL, B.VARIANT_TEMPORAL_WG4,
                                     B.VARIANT_TEMPORAL_WG8])
def test_temporal_fd8_matches_oracle(variant):
    ny, nx = 48, 70
    sch = schemes.ORDER8_K6
    steps, c = oracle_weights(sch)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / nx, 2, workloads.SIGMA_FD8)
    y0 = np.random.default_rng(4).standard_normal((3, ny, nx))
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, fd_order=8, check_stability=False)
    plan.set_variant(variant)
    got = plan.step(to_dev(y0[None]), n_macro=3).cpu().numpy()[0]
    want = G.integrate(OP.Acoustic((ny, nx), c2=1.0, r=4), 0.0, y0, H, 3, steps, c)
    assert rel_err(got, want, 0) <= TOL64


def test_fp32_stepping_error_vs_fp64():
    # FP32 levels, FP64 averaging and combination.  Stated bound for 20
    # macro steps on a 128^2 grid: max rel error <= 2e-5 (measured ~ 2-5e-6;
    # the scale is u32 * sum|c| * sqrt(number of rounding steps)).
    n = 128
    sch = schemes.ORDER8_K6
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / n, 2, workloads.SIGMA_FD4)
    y0 = fields.acoustic2d_pulse_modes(n, n_modes=8, kmax=6, width=0.05, seed=4)
    p64 = lib_plan(B.ACOUSTIC2D, (n, n), sch, H)
    p32 = lib_plan(B.ACOUSTIC2D, (n, n), sch, H, dtype=torch.float32)
    a = p64.step(to_dev(y0[None]), n_macro=20).cpu().numpy()
    b = p32.step(to_dev(y0[None], torch.float32), n_macro=20).cpu().numpy()
    err = rel_err(b, a, 1)
    print("fp32 vs fp64 rel err", err)
    assert err <= 2e-5


def test_acoustic2d_full_size_500_steps_vs_closed_form():
    # the benchmark's workload at full size and length, in the same launch
    # configuration; the constant-c closed form gives every grid value
    cfg = workloads.CONFIG_ACOUSTIC2D
    n = cfg["n"]
    steps, c = oracle_weights(cfg["scheme"])
    y0 = fields.acoustic2d_pulse_modes(n)
    plan = lib_plan(B.ACOUSTIC2D, (n, n), cfg["scheme"], cfg["H"])
    y = to_dev(y0[None])
    # the configuration bench.py times: autotuned on one lane
    tuned = plan.autotune(y, torch.empty_like(y), macro_steps=5, lanes=1)
    print("autotuned (variant, band, lanes)", tuned)
    out = plan.step(y, n_macro=cfg["n_macro"])
    got = out.cpu().numpy()[0]
    want = SP.acoustic(y0, 1.0, cfg["H"], steps, c, cfg["n_macro"])
    errs = [rel_err(got[q], want[q], None) for q in range(3)]
    print("full-size rel errors", errs)
    assert max(errs) <= TOL64


def test_plan_autotune_keeps_a_blocked_variant_with_the_same_result():
    ny, nx = 160, 120
    sch = schemes.ORDER8_K6
    cs = fields.lognormal_speed((ny, nx), seed=5)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    y0 = to_dev(np.random.default_rng(6).standard_normal((1, 3, ny, nx)))
    ref = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, c2_field=to_dev(cs ** 2), c_max=float(cs.max()))
    ref.set_variant(B.VARIANT_FLAT)
    want = ref.step(y0, n_macro=2).cpu().numpy()
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, c2_field=to_dev(cs ** 2), c_max=float(cs.max()))
    v, band, lanes = plan.autotune(y0, macro_steps=2)
    assert lanes in (1, 2, 3)
    assert v in (B.VARIANT_TEMPORAL, B.VARIANT_TEMPORAL4, B.VARIANT_TEMPORAL_S5,
                 B.VARIANT_TEMPORAL_S6, B.VARIANT_TEMPORAL_WG4, B.VARIANT_TEMPORAL_WG8)
    assert band in (0, 32, 64, 96, 128)
    assert plan.variant() == v
    got = plan.step(y0, n_macro=2).cpu().numpy()
    assert rel_err(got, want, 1) <= 1e-13


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_lanes_do_not_change_the_result(dtype):
    # the blocked passes spread over 1..4 streams compute the same values
    ny, nx = 150, 130
    sch = schemes.ORDER8_K6
    cs = fields.lognormal_speed((ny, nx), seed=8)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    y0 = to_dev(np.random.default_rng(9).standard_normal((2, 3, ny, nx)), dtype)
    s = fields.ricker_source_2d(max(nx, ny), cells_per_wavelength=8.0)
    outs = []
    for lanes in (1, 2, 3, 4):
        plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, n_rhs=2, dtype=dtype,
                        c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()))
        plan.set_sources([0], [60 * nx + 70], [s["weight"] * 1e-4], s["f0"], s["delay"])
        plan.set_lanes(lanes)
        outs.append(plan.step(y0, t0=0.3 * s["delay"], n_macro=4))
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


# Several point sources through the temporally blocked passes: two in one
# grid column of right-hand side 0 (rows 20 and 61), a third at the first
# one's point, a fourth in another column of the same 64-column strip, and
# one in right-hand side 1.  (rhs, (iy, ix), weight factor)
MULTI_SOURCES = [(0, (20, 30), 1.0), (0, (61, 30), -0.7), (0, (20, 30), 0.4),
                 (0, (45, 33), 0.9), (1, (50, 90), 1.3)]


def multi_source_problem(dtype=torch.float64):
    ny, nx = 90, 100
    cs = fields.lognormal_speed((ny, nx), seed=22)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    s = fields.ricker_source_2d(max(nx, ny), cells_per_wavelength=6.0)
    w0 = s["weight"] * 1e-3
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), schemes.ORDER8_K6, H, n_rhs=2, dtype=dtype,
                    c2_field=to_dev(c2, dtype), c_max=float(cs.max()))
    plan.set_sources([r for r, _, _ in MULTI_SOURCES],
                     [iy * nx + ix for _, (iy, ix), _ in MULTI_SOURCES],
                     [w0 * k for _, _, k in MULTI_SOURCES], s["f0"], s["delay"])
    ops = [OP.Acoustic((ny, nx), c2=c2, r=2,
                       sources=[OP.Source(idx, s["f0"], s["delay"], w0 * k)
                                for rr, idx, k in MULTI_SOURCES if rr == r])
           for r in range(2)]
    t0 = s["delay"] - 2 * H               # the wavelet near its peak
    return plan, ops, H, t0


@pytest.mark.parametrize("variant", [B.VARIANT_AUTO, B.VARIANT_TEMPORAL_S5, B.VARIANT_TEMPORAL,
                                     B.VARIANT_FLAT])
def test_blocked_passes_with_several_sources_vs_oracle(variant):
    plan, ops, H, t0 = multi_source_problem()
    steps, c = oracle_weights(schemes.ORDER8_K6)
    plan.set_variant(variant)
    rng = np.random.default_rng(23)
    y0 = 1e-3 * rng.standard_normal((2, 3) + ops[0].shape)
    got = plan.step(to_dev(y0), t0=t0, n_macro=3).cpu().numpy()
    for r in range(2):
        want = G.integrate(ops[r], t0, y0[r], H, 3, steps, c)
        assert rel_err(got[r], want, 0) <= TOL64, r


def test_plan_follows_torchs_current_stream():
    # a plan created on one stream and called under another enqueues on the
    # current one (ordered after the old one's work), with the same results
    n = 96
    sch = schemes.ORDER8_K6
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / n, 2, workloads.SIGMA_FD4)
    y0 = to_dev(np.random.default_rng(10).standard_normal((1, 3, n, n)))
    plan = lib_plan(B.ACOUSTIC2D, (n, n), sch, H)
    want = plan.step(y0, n_macro=3)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        got = plan.step(y0, n_macro=3)
        assert plan.stream.cuda_stream == s.cuda_stream
        got2 = plan.step(got, n_macro=2)
    torch.cuda.current_stream().wait_stream(s)
    assert torch.equal(got, want)
    back = plan.step(want, n_macro=2)
    assert plan.stream.cuda_stream == torch.cuda.current_stream().cuda_stream
    assert torch.equal(back, got2)


@pytest.mark.parametrize("variant", [B.VARIANT_TEMPORAL_S5, B.VARIANT_TEMPORAL])
@pytest.mark.parametrize("form", [B.FORM_SHARED_F0, B.FORM_FUSED_COMBINE,
                                  B.FORM_SHARED_F0 | B.FORM_FUSED_COMBINE,
                                  B.FORM_ALIGNED_FIRST,
                                  B.FORM_ALIGNED_FIRST | B.FORM_SHARED_F0])
def test_pass_forms_vs_oracle(form, variant):
    # f(t0, y0) shared by the first passes (Sect. 3.6), the combination
    # folded into the last sequence's final pass, and the first passes on one
    # strip geometry: the oracle's values (with the five sources of the
    # multi-source problem, c^2 field, two right-hand sides) and the default
    # form's to rounding
    plan, ops, H, t0 = multi_source_problem()
    steps, c = oracle_weights(schemes.ORDER8_K6)
    plan.set_variant(variant)
    y0 = 1e-3 * np.random.default_rng(25).standard_normal((2, 3) + ops[0].shape)
    ref = plan.step(to_dev(y0), t0=t0, n_macro=3).cpu().numpy()
    plan.set_form(form)
    got = plan.step(to_dev(y0), t0=t0, n_macro=3).cpu().numpy()
    for r in range(2):
        want = G.integrate(ops[r], t0, y0[r], H, 3, steps, c)
        assert rel_err(got[r], want, 0) <= TOL64, r
    assert rel_err(got, ref, 1) <= 1e-13


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("variant,order", [(B.VARIANT_TEMPORAL_S5, 0), (B.VARIANT_TEMPORAL4, 0),
                                           (B.VARIANT_TEMPORAL, 0), (B.VARIANT_TEMPORAL_S5, 1)])
def test_aligned_first_passes_equal_the_default(dtype, variant, order):
    # every column's value comes from the same arithmetic whichever strip
    # and lane compute it, so the first passes on the widest halo's strip
    # geometry (wider recomputed halo for the passes with fewer evaluations,
    # 3 strips of 44 columns for 100, sources in several columns) change no
    # bit; with the hardware order or another workgroup order as well
    plan, ops, H, t0 = multi_source_problem(dtype)
    plan.set_variant(variant)
    y0 = to_dev(1e-3 * np.random.default_rng(29).standard_normal((2, 3) + ops[0].shape), dtype)
    ref = plan.step(y0, t0=t0, n_macro=2)
    plan.set_form(B.FORM_ALIGNED_FIRST)
    plan.set_wave_order(order)
    got = plan.step(y0, t0=t0, n_macro=2)
    assert torch.equal(got, ref)


@pytest.mark.parametrize("order", [1, 2])
def test_wave_orders_do_not_change_the_result(order):
    plan, ops, H, t0 = multi_source_problem()
    y0 = to_dev(1e-3 * np.random.default_rng(26).standard_normal((2, 3) + ops[0].shape))
    ref = plan.step(y0, t0=t0, n_macro=2)
    plan.set_wave_order(order)
    got = plan.step(y0, t0=t0, n_macro=2)
    assert torch.equal(got, ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(70, 22, 90), (64, 32, 128), (9, 9, 9), (130, 64, 128)])
def test_tile3d_matches_flat_and_oracle(dtype, shape):
    # the LDS-tiled 3-D sweeps against the one-point-per-thread ones (the same
    # stencil sums; products may contract differently) and, for the ragged
    # grid, against the oracle; ragged tiles in x, y and z, the smallest grid
    # FD8 allows, smaller than one tile, and a grid of 16 tiles (a multiple
    # of 8: the XCD-grouped orders of tiles and of each tile's sequences)
    nz, ny, nx = shape
    cs = fields.lognormal_speed(shape, seed=27)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(shape), 3,
                           workloads.SIGMA_FD8)
    y0 = np.random.default_rng(28).standard_normal((2, 4) + shape)
    srcs = [(0, (nz // 2, ny // 3, nx // 4), 1e3), (1, (0, 0, 7), -5e2)]
    outs = []
    for v in (B.VARIANT_FLAT, B.VARIANT_TILE3D):
        plan = lib_plan(B.ACOUSTIC3D, (nx, ny, nz), schemes.ORDER8_K6, H, fd_order=8, n_rhs=2,
                        dtype=dtype, c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()),
                        check_stability=False)
        plan.set_sources([r for r, _, _ in srcs], [(z * ny + y) * nx + x for _, (z, y, x), _ in srcs],
                         [w for _, _, w in srcs], 25.0, 0.004)
        plan.set_variant(v)
        outs.append(plan.step(to_dev(y0, dtype), t0=0.003, n_macro=2).double().cpu().numpy())
    e = rel_err(outs[1], outs[0], 1)
    print(shape, dtype, "tile3d vs flat", e)
    assert e <= (1e-13 if dtype == torch.float64 else 2e-6)
    if shape == (70, 22, 90):
        steps, c = oracle_weights(schemes.ORDER8_K6)
        for r, idx, w in srcs:
            op = OP.Acoustic(shape, c2=cs ** 2, r=4, sources=[OP.Source(idx, 25.0, 0.004, w)])
            want = G.integrate(op, 0.003, y0[r], H, 2, steps, c)
            e = rel_err(outs[1][r], want, 0)
            print("tile3d vs oracle, rhs", r, e)
            assert e <= (TOL64 if dtype == torch.float64 else 3e-5)
