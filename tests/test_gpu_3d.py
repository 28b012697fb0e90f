"""The 3-D FD8 multi-right-hand-side workload at the parity grid (96^3, the
384^3 field sampled every 4th point, the same 8 source positions): FP64
against the oracle, FP32 stepping against the oracle with a stated bound,
the right-hand sides of one batched plan against single-source plans, and
the adjoint against the oracle's discrete adjoint; and at its full size
(384^3, 8 right-hand sides, the benchmark's launch configuration), sampled
outputs against the oracle on periodic windows around them."""
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
        e64 = rel_err(out[torch.float64][r], want, 0)
        e32 = rel_err(out[torch.float32][r], want, 0)
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
    assert rel_err(res[torch.float64][0], want_y, 0) <= TOL64
    assert rel_err(res[torch.float64][1], want_g, None) <= TOL64
    e_y = rel_err(res[torch.float32][0], want_y, 0)
    e_g = rel_err(res[torch.float32][1], want_g, None)
    print("fp32 adjoint vs oracle: ybar", e_y, "grad", e_g)
    assert e_y <= TOL32 and e_g <= TOL32


# FP32 stepping over the 6 macro steps of the gradient test: the worst-case
# linear growth of the one-step bound above, 6 * 3e-5, rounded up
TOL32_GRAD = 2e-4


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_acoustic3d_checkpointed_gradient_vs_oracle(dtype):
    # the 3-D differentiation path at a size the oracle finishes in seconds:
    # 24^3 FD8, log-normal c^2, two right-hand sides (one Ricker source
    # each), 16 receivers per right-hand side on z planes, 6 macro steps,
    # checkpoints every 2; L, dL/dy0 and dL/dc^2 against the oracle
    from paper_1907_11771_amd.autograd import receiver_traces
    n, n_macro = 24, 6
    cs = fields.lognormal_speed((n, n, n), seed=62)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / n, 3, workloads.SIGMA_FD8)
    steps, c = oracle_weights(schemes.ORDER8_K6)
    pts = [(5, 12, 7), (17, 4, 19)]
    src = fields.ricker_source_3d(n, pts, cells_per_wavelength=6.0)
    w = src["weight"] * 1e-3
    recs = [np.array(fields.plane_receivers_3d(n, count=16, z=2)),
            np.array(fields.plane_receivers_3d(n, count=16, z=20))]
    plan = lib_plan(B.ACOUSTIC3D, (n, n, n), schemes.ORDER8_K6, H, fd_order=8, n_rhs=2,
                    dtype=dtype, c2_field=to_dev(c2, dtype), c_max=float(cs.max()))
    plan.set_sources([0, 1], [z * n * n + y * n + x for z, y, x in pts], [w, w],
                     src["f0"], src["delay"])
    plan.set_receivers([r for r in range(2) for _ in recs[r]],
                       [int(z) * n * n + int(y) * n + int(x) for rr in recs for z, y, x in rr])
    rng = np.random.default_rng(63)
    y0 = np.zeros((2, 4, n, n, n))
    for r in range(2):
        y0[r, 0] = 1e-2 * fields.gaussian_random_field((n, n, n), ell=0.15, seed=64 + r)
    data = [1e-3 * rng.standard_normal((n_macro, len(rr))) for rr in recs]
    t0 = 0.5 * src["delay"]
    y = to_dev(y0, dtype).requires_grad_(True)
    c2t = plan.c2_field.clone().requires_grad_(True)
    tr = receiver_traces(plan, y, c2t, n_macro, t0=t0, checkpoint_every=2)
    loss = 0.5 * ((tr.double() - to_dev(np.concatenate(data, axis=1))) ** 2).sum()
    loss.backward()
    ops = [OP.Acoustic((n, n, n), c2=c2, r=4,
                       sources=[OP.Source(p, src["f0"], src["delay"], w)]) for p in pts]
    L, gys, gc = AD.misfit_gradient_rhs(ops, t0, list(y0), H, steps, c, n_macro, recs, data)
    e_l = abs(float(loss.detach()) - L) / L
    e_y = max(rel_err(y.grad.double().cpu().numpy()[r], gys[r], 0) for r in range(2))
    e_g = rel_err(c2t.grad.double().cpu().numpy(), gc, None)
    print(dtype, "3-D gradient vs oracle: L", e_l, "dL/dy0", e_y, "dL/dc2", e_g)
    tol = 1e-11 if dtype == torch.float64 else TOL32_GRAD
    assert e_l <= tol and e_y <= tol and e_g <= tol


def test_full_size_384_eight_rhs_sampled_windows_vs_oracle():
    # the 384^3 workload itself, in the launch configuration the benchmark
    # times (one plan, all 8 right-hand sides with their sources, the
    # LDS-tiled sweeps, FP32 stepping and FP64), one macro step, sampled: the
    # oracle runs on periodic windows of half-width 56 around two points,
    # with the full grid's spacing, and is exact at the 9^3 points within 4
    # of each window's middle (the longest sequence's 13 evaluations reach
    # 13 x 4 = 52 points).  The input is random inside the two windows (right-
    # hand side 0 around its source, right-hand side 5 across the periodic
    # boundary) and zero elsewhere.
    cfg = workloads.CONFIG_3D
    n, R = cfg["n"], cfg["n_rhs"]
    hw, k = 56, 4
    steps, c = oracle_weights(schemes.ORDER8_K6)
    cs = fields.bandlimited_lognormal_speed(n, seed=cfg["speed_seed"], kmax=cfg["kmax"])
    c2 = cs ** 2
    cmax = float(cs.max())
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cmax, 1.0 / n, 3, workloads.SIGMA_FD8)
    src = fields.ricker_source_3d(n, workloads.sources_3d(n, R, cfg["source_seed"]))
    t0 = src["delay"] - 0.5 * H
    rng = np.random.default_rng(63)
    centres = {0: tuple(p + d for p, d in zip(src["points"][0], (3, -2, 1))),
               5: (2, n - 3, n // 2)}
    blocks = {r: rng.standard_normal((4,) + (2 * hw + 1,) * 3) for r in centres}
    idx = {r: [np.arange(q - hw, q + hw + 1) % n for q in ctr] for r, ctr in centres.items()}
    # the oracle on each window (its own source where it lies inside)
    want = {}
    for r, (iz, iy, ix) in idx.items():
        lo = [q - hw for q in centres[r]]
        local = [tuple((p - l) % n for p, l in zip(src["points"][r], lo))]
        local = [q for q in local if all(v <= 2 * hw for v in q)]
        op = OP.Acoustic((2 * hw + 1,) * 3, c2=c2[np.ix_(iz, iy, ix)], r=4,
                         spacing=(1.0 / n,) * 3,
                         sources=[OP.Source(q, src["f0"], src["delay"], src["weight"])
                                  for q in local])
        full = G.macro_step(op, t0, blocks[r], H, steps, c)
        want[r] = full[:, hw - k:hw + k + 1, hw - k:hw + k + 1, hw - k:hw + k + 1]
    for dtype, tol in ((torch.float32, TOL32), (torch.float64, TOL64)):
        y = torch.zeros((R, 4, n, n, n), dtype=dtype, device="cuda")
        for r, (iz, iy, ix) in idx.items():
            tz, ty, tx = [torch.from_numpy(a).cuda() for a in (iz, iy, ix)]
            y[r][:, tz[:, None, None], ty[None, :, None], tx[None, None, :]] = \
                torch.from_numpy(blocks[r]).to("cuda", dtype)
        plan = lib_plan(B.ACOUSTIC3D, (n, n, n), schemes.ORDER8_K6, H, fd_order=8, n_rhs=R,
                        dtype=dtype, c2_field=to_dev(c2, dtype), c_max=cmax)
        assert plan.variant() == B.VARIANT_TILE3D
        plan.set_sources(list(range(R)), [z * n * n + yy * n + x for z, yy, x in src["points"]],
                         [src["weight"]] * R, src["f0"], src["delay"])
        plan.step(y, out=y, t0=t0, n_macro=1)
        for r, (iz, iy, ix) in idx.items():
            tz, ty, tx = [torch.from_numpy(a[hw - k:hw + k + 1]).cuda() for a in (iz, iy, ix)]
            got = y[r][:, tz[:, None, None], ty[None, :, None], tx[None, None, :]]
            e = rel_err(got.double().cpu().numpy(), want[r], 0)
            print("384^3", dtype, "rhs", r, "vs oracle window", e, flush=True)
            assert e <= tol, (dtype, r, e)
        del plan, y
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
