"""GPU adjoint: one macro step against the oracle's discrete adjoint, the
dot-product identity with the library's own forward step, the checkpointed
misfit gradient against the oracle, and central differences at the full
size of the differentiation workload."""
import numpy as np
import pytest
import torch

from oracle import adjoint as AD
from oracle import operators as OP
from paper_1907_11771_amd import binding as B
from paper_1907_11771_amd.autograd import receiver_traces
from synth import fields, schemes, workloads
from tests.gpu_util import lib_plan, oracle_weights, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _setup2d(nx=40, ny=32, source=True, dtype=torch.float64):
    sch = schemes.ORDER8_K6
    cs = fields.lognormal_speed((ny, nx), seed=31)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), sch, H, c2_field=to_dev(c2, dtype),
                    c_max=float(cs.max()), dtype=dtype)
    srcs = []
    if source:
        s = fields.ricker_source_2d(max(nx, ny), cells_per_wavelength=6.0)
        w = s["weight"] * 1e-3
        plan.set_sources([0], [(ny // 2) * nx + nx // 3], [w], s["f0"], s["delay"])
        srcs = [OP.Source((ny // 2, nx // 3), s["f0"], s["delay"], w)]
    op = OP.Acoustic((ny, nx), c2=c2, r=2, sources=srcs)
    return plan, op, H


def test_adjoint_macro_step_matches_oracle():
    plan, op, H = _setup2d()
    steps, c = oracle_weights(schemes.ORDER8_K6)
    rng = np.random.default_rng(0)
    y0 = rng.standard_normal((3,) + op.shape)
    wbar = rng.standard_normal((3,) + op.shape)
    t0 = 0.01
    ybar = to_dev(wbar[None])
    grad = torch.zeros(op.shape, dtype=torch.float64, device="cuda")
    plan.adjoint_step(t0, to_dev(y0[None]), ybar, grad_c2=grad)
    want_y, want_g = AD.macro_step_adjoint(op, t0, y0, H, steps, c, wbar)
    assert rel_err(ybar.cpu().numpy()[0], want_y, 0) <= 1e-12
    assert rel_err(grad.cpu().numpy(), want_g, None) <= 1e-12


def test_adjoint_3d_fd8_two_rhs_matches_oracle():
    shape = (10, 12, 14)
    cs = fields.lognormal_speed(shape, seed=8)
    c2 = cs ** 2
    sch = schemes.ORDER8_K6
    steps, c = oracle_weights(sch)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / 14, 3, workloads.SIGMA_FD8)
    plan = lib_plan(B.ACOUSTIC3D, (14, 12, 10), sch, H, fd_order=8, n_rhs=2,
                    c2_field=to_dev(c2), c_max=float(cs.max()))
    rng = np.random.default_rng(1)
    y0 = rng.standard_normal((2, 4) + shape)
    wbar = rng.standard_normal((2, 4) + shape)
    ybar = to_dev(wbar)
    grad = torch.zeros(shape, dtype=torch.float64, device="cuda")
    plan.adjoint_step(0.0, to_dev(y0), ybar, grad_c2=grad)
    op = OP.Acoustic(shape, c2=c2, r=4)
    g_total = np.zeros(shape)
    for r in range(2):
        wy, wg = AD.macro_step_adjoint(op, 0.0, y0[r], H, steps, c, wbar[r])
        assert rel_err(ybar.cpu().numpy()[r], wy, 0) <= 1e-12
        g_total += wg
    assert rel_err(grad.cpu().numpy(), g_total, None) <= 1e-12


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13), (torch.float32, 1e-5)])
def test_dot_product_identity_with_library_forward(dtype, tol):
    plan, op, H = _setup2d(source=False, dtype=dtype)
    rng = np.random.default_rng(2)
    d = to_dev(rng.standard_normal((1, 3) + op.shape), dtype)
    w = to_dev(rng.standard_normal((1, 3) + op.shape), dtype)
    fwd = plan.step(d, n_macro=1)
    adj = w.clone()
    plan.adjoint_step(0.0, d, adj)
    lhs = float((fwd.double() * w.double()).sum())
    rhs = float((d.double() * adj.double()).sum())
    assert abs(lhs - rhs) <= tol * max(abs(lhs), 1.0)


@pytest.mark.parametrize("duplicate", [False, True])
def test_checkpointed_misfit_gradient_matches_oracle(duplicate):
    plan, op, H = _setup2d(nx=32, ny=24)
    steps, c = oracle_weights(schemes.ORDER8_K6)
    nx, ny = 32, 24
    rec = fields.edge_receivers_2d(nx, count=8, row=3)
    if duplicate:
        # two receivers at one point: their adjoints are injected in order
        rec = np.concatenate([rec, rec[2:3]])
    plan.set_receivers([0] * len(rec), [int(r[0]) * nx + int(r[1]) for r in rec])
    n_macro = 7
    y0 = fields.acoustic2d_pulse_modes(nx, n_modes=4, kmax=3, width=0.1, seed=7)[:, :ny, :]
    data = np.random.default_rng(3).standard_normal((n_macro, len(rec))) * 1e-2
    y = to_dev(y0[None]).requires_grad_(True)
    c2 = plan.c2_field.clone().requires_grad_(True)
    tr = receiver_traces(plan, y, c2, n_macro, t0=0.0, checkpoint_every=3)
    loss = 0.5 * ((tr - to_dev(data)) ** 2).sum()
    loss.backward()
    L, gy, gc = AD.misfit_gradient(op, 0.0, y0, H, steps, c, n_macro, rec, data)
    assert float(loss.detach()) == pytest.approx(L, rel=1e-12)
    assert rel_err(y.grad.cpu().numpy()[0], gy, 0) <= 1e-11
    assert rel_err(c2.grad.cpu().numpy(), gc, None) <= 1e-11


def test_full_size_gradient_vs_central_differences():
    # the differentiation workload: 1024^2, log-normal c^2, one Ricker source,
    # 128 receivers on one row, 400 macro steps, checkpoints every 20; data
    # from a run with a perturbed c^2; FP64
    n, n_macro = 1024, 400
    sch = schemes.ORDER8_K6
    cs = fields.lognormal_speed((n, n), seed=40)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / n, 2, workloads.SIGMA_FD4)
    plan = lib_plan(B.ACOUSTIC2D, (n, n), sch, H, c2_field=to_dev(c2), c_max=float(cs.max()) * 1.01)
    s = fields.ricker_source_2d(n)
    plan.set_sources([0], [s["idx"][0] * n + s["idx"][1]], [s["weight"]], s["f0"], s["delay"])
    rec = fields.edge_receivers_2d(n, count=128)
    plan.set_receivers([0] * 128, [int(r[0]) * n + int(r[1]) for r in rec])
    y0 = torch.zeros((1, 3, n, n), dtype=torch.float64, device="cuda")
    c2_obs = to_dev(c2 * np.exp(0.1 * fields.gaussian_random_field((n, n), seed=41)))
    with torch.no_grad():
        data = receiver_traces(plan, y0, c2_obs, n_macro)
    c2d = to_dev(c2)

    def loss_of(c2v, y0v):
        return 0.5 * ((receiver_traces(plan, y0v, c2v, n_macro) - data) ** 2).sum()

    c2v = c2d.clone().requires_grad_(True)
    y0v = y0.clone().requires_grad_(True)
    loss = loss_of(c2v, y0v)
    loss.backward()
    g = c2v.grad
    gy = y0v.grad
    with torch.no_grad():
        for k in range(16):
            dirn = to_dev(fields.gaussian_random_field((n, n), ell=0.15, seed=500 + k)) * c2d
            dirn = dirn / dirn.norm()
            # central differences at eps and eps/2, Richardson-extrapolated
            # (error O(eps^4)); eps is 2e-5 of the field's size
            eps = 2e-5 * float(c2d.norm())
            fds = []
            for e in (eps, eps / 2):
                lp = float(loss_of(c2d + e * dirn, y0))
                lm = float(loss_of(c2d - e * dirn, y0))
                fds.append((lp - lm) / (2 * e))
            fd = (4 * fds[1] - fds[0]) / 3
            ad = float((g * dirn).sum())
            assert ad == pytest.approx(fd, rel=1e-6), (k, ad, fds)
        # the misfit is quadratic in p(0): central differences are exact
        dp = torch.zeros_like(y0)
        dp[0, 0] = to_dev(fields.gaussian_random_field((n, n), ell=0.05, seed=600))
        eps = 1e-3
        fd = (float(loss_of(c2d, y0 + eps * dp)) - float(loss_of(c2d, y0 - eps * dp))) / (2 * eps)
        ad = float((gy * dp).sum())
        assert ad == pytest.approx(fd, rel=1e-7)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-14), (torch.float32, 1e-6)])
@pytest.mark.parametrize("shape", [(70, 22, 90), (130, 64, 128)])
def test_adjoint_3d_march_matches_flat(dtype, tol, shape):
    # the z-marching adjoint sweeps against the flat ones: same products and
    # sums (the gradient adds the right-hand sides one at a time), ragged
    # against the 64 x 4 x 64 tiles; the second grid has a multiple of 8
    # tiles in every tiled form (the XCD-grouped tile orders) and a ragged
    # last z chunk
    nz, ny, nx = shape
    cs = fields.lognormal_speed(shape, seed=14)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(shape), 3,
                           workloads.SIGMA_FD8)
    rng = np.random.default_rng(15)
    y0 = to_dev(rng.standard_normal((2, 4) + shape), dtype)
    wbar = rng.standard_normal((2, 4) + shape)
    res = []
    for v in (B.VARIANT_FLAT, B.VARIANT_MARCH8, B.VARIANT_TILE3D):
        plan = lib_plan(B.ACOUSTIC3D, (nx, ny, nz), schemes.ORDER8_K6, H, fd_order=8, n_rhs=2,
                        dtype=dtype, c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()))
        plan.set_sources([0], [(30 * ny + 5) * nx + 7], [1e3], 25.0, 0.004)
        plan.set_variant(v)
        ybar = to_dev(wbar, dtype)
        grad = torch.zeros(shape, dtype=torch.float64, device="cuda")
        plan.adjoint_step(0.003, y0, ybar, grad_c2=grad)
        res.append((ybar.double().cpu().numpy(), grad.cpu().numpy()))
    assert rel_err(res[1][0], res[0][0], 1) <= tol
    assert rel_err(res[1][1], res[0][1], None) <= tol
    # the LDS-tiled forward sweeps in the recomputation of the levels
    assert rel_err(res[2][0], res[0][0], 1) <= 10 * tol
    assert rel_err(res[2][1], res[0][1], None) <= 10 * tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
@pytest.mark.parametrize("band", [64, 19, 0])
def test_blocked_adjoint_matches_streaming(dtype, tol, band):
    # the temporally blocked adjoint (levels regenerated backwards, Psi
    # variables) against the streaming one (levels stored), two right-hand
    # sides with a source, ragged against strips and bands
    ny, nx = 150, 130
    cs = fields.lognormal_speed((ny, nx), seed=16)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    rng = np.random.default_rng(17)
    y0 = to_dev(rng.standard_normal((2, 3, ny, nx)), dtype)
    wbar = rng.standard_normal((2, 3, ny, nx))
    s = fields.ricker_source_2d(max(nx, ny), cells_per_wavelength=6.0)
    res = []
    for v in (B.VARIANT_FLAT, B.VARIANT_TEMPORAL):
        plan = lib_plan(B.ACOUSTIC2D, (nx, ny), schemes.ORDER8_K6, H, n_rhs=2, dtype=dtype,
                        c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()))
        plan.set_sources([1], [70 * nx + 40], [s["weight"] * 1e-3], s["f0"], s["delay"])
        plan.set_variant(v)
        B.check(B.lib().gbs_plan_set_band(plan.handle, band))
        ybar = to_dev(wbar, dtype)
        grad = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
        plan.adjoint_step(0.9 * s["delay"], y0, ybar, grad_c2=grad)
        res.append((ybar.double().cpu().numpy(), grad.cpu().numpy()))
    assert rel_err(res[1][0], res[0][0], 1) <= tol
    assert rel_err(res[1][1], res[0][1], None) <= tol


def test_blocked_adjoint_lanes_do_not_change_the_result():
    ny, nx = 150, 130
    cs = fields.lognormal_speed((ny, nx), seed=18)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    rng = np.random.default_rng(19)
    y0 = to_dev(rng.standard_normal((1, 3, ny, nx)))
    wbar = rng.standard_normal((1, 3, ny, nx))
    s = fields.ricker_source_2d(max(nx, ny), cells_per_wavelength=6.0)
    res = []
    for lanes in (1, 3):
        plan = lib_plan(B.ACOUSTIC2D, (nx, ny), schemes.ORDER8_K6, H, c2_field=to_dev(cs ** 2),
                        c_max=float(cs.max()))
        plan.set_sources([0], [70 * nx + 40], [s["weight"] * 1e-3], s["f0"], s["delay"])
        plan.set_lanes(lanes)
        ybar = to_dev(wbar)
        grad = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
        plan.adjoint_step(0.9 * s["delay"], y0, ybar, grad_c2=grad)
        res.append((ybar.clone(), grad.clone()))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("variant,lanes", [(B.VARIANT_TEMPORAL_S5, 1), (B.VARIANT_TEMPORAL, 2)])
def test_kept_pairs_give_the_same_adjoint(dtype, variant, lanes):
    # the forward step that keeps (y_{N-1}, y_N) returns the same state, and
    # the adjoint from the kept levels equals the one that rebuilds them
    ny, nx = 150, 130
    cs = fields.lognormal_speed((ny, nx), seed=20)
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                           workloads.SIGMA_FD4)
    rng = np.random.default_rng(21)
    y0 = to_dev(rng.standard_normal((2, 3, ny, nx)), dtype)
    wbar = rng.standard_normal((2, 3, ny, nx))
    s = fields.ricker_source_2d(max(nx, ny), cells_per_wavelength=6.0)
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), schemes.ORDER8_K6, H, n_rhs=2, dtype=dtype,
                    c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()))
    plan.set_sources([1], [70 * nx + 40], [s["weight"] * 1e-3], s["f0"], s["delay"])
    plan.set_variant(variant)
    plan.set_lanes(lanes)
    t0 = 0.9 * s["delay"]
    n_macro = 3
    pairs = torch.empty(plan.pairs_shape(n_macro), dtype=dtype, device="cuda")
    y_keep = torch.empty_like(y0)
    plan.step_keep_pairs(y0, y_keep, pairs, t0=t0, n_macro=n_macro)
    states = [y0.clone()]
    for m in range(n_macro):
        states.append(plan.step(states[-1], t0=t0 + m * H))
    assert torch.equal(y_keep, states[-1])
    for m in range(n_macro):
        res = []
        for kept in (False, True):
            ybar = to_dev(wbar, dtype)
            grad = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
            if kept:
                plan.adjoint_step_pairs(t0 + m * H, states[m], pairs[m], ybar, grad_c2=grad)
            else:
                plan.adjoint_step(t0 + m * H, states[m], ybar, grad_c2=grad)
            res.append((ybar, grad))
        assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1]), m


def test_checkpointed_gradient_with_kept_pairs():
    plan, op, H = _setup2d(nx=64, ny=48)
    nx, ny = 64, 48
    rec = fields.edge_receivers_2d(nx, count=8, row=3)
    plan.set_receivers([0] * len(rec), [int(r[0]) * nx + int(r[1]) for r in rec])
    n_macro = 9
    y0 = fields.acoustic2d_pulse_modes(nx, n_modes=4, kmax=3, width=0.1, seed=8)[:, :ny, :]
    data = to_dev(np.random.default_rng(5).standard_normal((n_macro, len(rec))) * 1e-2)
    grads = []
    for keep, adj_lanes in ((False, None), (True, None), (True, 3)):
        plan.adjoint_lanes = adj_lanes
        y = to_dev(y0[None]).requires_grad_(True)
        c2 = plan.c2_field.clone().requires_grad_(True)
        tr = receiver_traces(plan, y, c2, n_macro, checkpoint_every=4, keep_pairs=keep)
        (0.5 * ((tr - data) ** 2).sum()).backward()
        grads.append((y.grad.clone(), c2.grad.clone()))
        assert plan.lanes == 1                        # the forward's lanes are restored
    for g in grads[1:]:
        assert torch.equal(grads[0][0], g[0]) and torch.equal(grads[0][1], g[1])
    assert plan.autotune_adjoint(to_dev(y0[None])) in (1, 2, 3)
    assert plan.lanes == 1


def test_kept_pairs_need_the_blocked_form():
    plan, _, _ = _setup2d()
    plan.set_variant(B.VARIANT_FLAT)
    y = torch.zeros(plan.state_shape, dtype=torch.float64, device="cuda")
    pairs = torch.empty(plan.pairs_shape(1), dtype=torch.float64, device="cuda")
    with pytest.raises(B.GBSError) as ei:
        plan.step_keep_pairs(y, y.clone(), pairs)
    assert ei.value.status == B.GBS_EUNSUPPORTED
    assert not plan.blocked_adjoint()


@pytest.mark.parametrize("variant", [B.VARIANT_AUTO, B.VARIANT_FLAT])
def test_adjoint_with_several_sources_vs_oracle(variant):
    # the blocked adjoint (and the streaming one) with sources sharing a
    # column, a point and a strip, in two right-hand sides
    from tests.test_gpu_parity import multi_source_problem
    plan, ops, H, t0 = multi_source_problem()
    plan.set_variant(variant)
    assert plan.blocked_adjoint() == (variant == B.VARIANT_AUTO)
    steps, c = oracle_weights(schemes.ORDER8_K6)
    rng = np.random.default_rng(24)
    y0 = rng.standard_normal((2, 3) + ops[0].shape)
    wbar = rng.standard_normal((2, 3) + ops[0].shape)
    ybar = to_dev(wbar)
    grad = torch.zeros(ops[0].shape, dtype=torch.float64, device="cuda")
    plan.adjoint_step(t0, to_dev(y0), ybar, grad_c2=grad)
    g_total = np.zeros(ops[0].shape)
    for r in range(2):
        wy, wg = AD.macro_step_adjoint(ops[r], t0, y0[r], H, steps, c, wbar[r])
        assert rel_err(ybar.cpu().numpy()[r], wy, 0) <= 1e-12, r
        g_total += wg
    assert rel_err(grad.cpu().numpy(), g_total, None) <= 1e-12


def test_backward_uses_its_own_forwards_c2():
    # a second forward with another c^2 between the first forward and its
    # backward (a line-search probe) must not change the first gradient
    plan, op, H = _setup2d(nx=32, ny=24)
    steps, c = oracle_weights(schemes.ORDER8_K6)
    nx = 32
    rec = fields.edge_receivers_2d(nx, count=8, row=3)
    plan.set_receivers([0] * len(rec), [int(r[0]) * nx + int(r[1]) for r in rec])
    n_macro = 5
    y0 = fields.acoustic2d_pulse_modes(nx, n_modes=4, kmax=3, width=0.1, seed=9)[:, :24, :]
    data = np.random.default_rng(6).standard_normal((n_macro, len(rec))) * 1e-2
    y = to_dev(y0[None]).requires_grad_(True)
    c2 = plan.c2_field.clone().requires_grad_(True)
    loss = 0.5 * ((receiver_traces(plan, y, c2, n_macro, checkpoint_every=2)
                   - to_dev(data)) ** 2).sum()
    c2b = (1.3 * plan.c2_field).requires_grad_(True)
    probe = 0.5 * ((receiver_traces(plan, y.detach(), c2b, n_macro) - to_dev(data)) ** 2).sum()
    loss.backward()
    L, gy, gc = AD.misfit_gradient(op, 0.0, y0, H, steps, c, n_macro, rec, data)
    assert float(loss.detach()) == pytest.approx(L, rel=1e-12)
    assert rel_err(y.grad.cpu().numpy()[0], gy, 0) <= 1e-11
    assert rel_err(c2.grad.cpu().numpy(), gc, None) <= 1e-11
    # and the probe's own backward still gives the probe's gradient
    probe.backward()
    op_b = OP.Acoustic(op.shape, c2=1.3 * op.c2, r=2, sources=op.sources)
    _, _, gcb = AD.misfit_gradient(op_b, 0.0, y0, H, steps, c, n_macro, rec, data)
    assert rel_err(c2b.grad.cpu().numpy(), gcb, None) <= 1e-11
