"""GPU parity at the edges of the input space: the smallest grids the
stencils admit (2R + 1 points along an axis, so that every stencil reaches
around the periodic box and a 64-lane strip covers the row several times),
grids minimal along one axis and long along another, the same through the
batch and the adjoint, and the zero state (a linear step of zero is zero,
exactly).  Every kernel variant that the operator admits runs, against the
oracle on the same seeded inputs (FP64 bar 1e-12 per field)."""
import numpy as np
import pytest
import torch

from oracle import adjoint as AD
from oracle import gbs as G
from oracle import operators as OP
from paper_1907_11771_amd import binding as B
from paper_1907_11771_amd.plan import GBSBatch, scheme_weights
from synth import fields, schemes, workloads
from tests.gpu_util import lib_plan, oracle_weights, rel_err, to_dev

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
SCH = schemes.ORDER8_K6

VARIANTS_FD4 = [B.VARIANT_FLAT, B.VARIANT_MARCH8, B.VARIANT_MARCH16_NT, B.VARIANT_PLAIN,
                B.VARIANT_TEMPORAL, B.VARIANT_TEMPORAL4, B.VARIANT_TEMPORAL_S5,
                B.VARIANT_TEMPORAL_S6, B.VARIANT_TEMPORAL_WG4, B.VARIANT_TEMPORAL_WG8]
VARIANTS_FD8 = [B.VARIANT_FLAT, B.VARIANT_MARCH8, B.VARIANT_PLAIN, B.VARIANT_TEMPORAL,
                B.VARIANT_TEMPORAL_WG4, B.VARIANT_TEMPORAL_WG8]
VARIANTS_3D = [B.VARIANT_FLAT, B.VARIANT_MARCH8, B.VARIANT_MARCH16, B.VARIANT_PLAIN,
               B.VARIANT_TILE3D]


def _acoustic2d(shape, r, seed):
    """Plan inputs for a (ny, nx) grid with a c^2 field and a Ricker source
    on the last grid point of right-hand side 1."""
    ny, nx = shape
    cs = fields.lognormal_speed((ny, nx), seed=seed)
    sig = workloads.SIGMA_FD4 if r == 2 else workloads.SIGMA_FD8
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2, sig)
    s = fields.ricker_source_2d(max(nx, ny), cells_per_wavelength=6.0)
    src = dict(idx=(ny - 1, nx - 1), f0=s["f0"], delay=s["delay"], w=s["weight"] * 1e-3)
    return cs ** 2, float(cs.max()), H, src


@pytest.mark.parametrize("variant", VARIANTS_FD4)
@pytest.mark.parametrize("shape", [(5, 5), (5, 131), (131, 5)], ids=["5x5", "5x131", "131x5"])
def test_acoustic2d_fd4_minimum_grids_vs_oracle(shape, variant):
    _check_2d(shape, 2, variant)


@pytest.mark.parametrize("variant", VARIANTS_FD8)
@pytest.mark.parametrize("shape", [(9, 9), (9, 140), (140, 9)], ids=["9x9", "9x140", "140x9"])
def test_acoustic2d_fd8_minimum_grids_vs_oracle(shape, variant):
    _check_2d(shape, 4, variant)


def _check_2d(shape, r, variant):
    ny, nx = shape
    steps, c = oracle_weights(SCH)
    c2, cmax, H, src = _acoustic2d(shape, r, seed=ny * 1000 + nx)
    y0 = np.random.default_rng(ny + 7 * nx).standard_normal((2, 3, ny, nx))
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), SCH, H, fd_order=2 * r, n_rhs=2,
                    c2_field=to_dev(c2), c_max=cmax)
    (iy, ix) = src["idx"]
    plan.set_sources([1], [iy * nx + ix], [src["w"]], src["f0"], src["delay"])
    plan.set_variant(variant)
    t0 = 0.4 * src["delay"]
    got = plan.step(to_dev(y0), t0=t0, n_macro=3).cpu().numpy()
    for rhs in range(2):
        srcs = [OP.Source(src["idx"], src["f0"], src["delay"], src["w"])] if rhs == 1 else []
        op = OP.Acoustic((ny, nx), c2=c2, r=r, sources=srcs)
        want = G.integrate(op, t0, y0[rhs], H, 3, steps, c)
        assert rel_err(got[rhs], want, 0) <= TOL64, rhs


@pytest.mark.parametrize("variant", VARIANTS_3D)
@pytest.mark.parametrize("shape", [(9, 9, 9), (9, 9, 70), (70, 9, 9), (9, 70, 9)],
                         ids=["9x9x9", "9x9x70", "70x9x9", "9x70x9"])
def test_acoustic3d_fd8_minimum_grids_vs_oracle(shape, variant):
    nz, ny, nx = shape
    steps, c = oracle_weights(SCH)
    cs = fields.lognormal_speed(shape, seed=nz + 3 * ny + 5 * nx)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(shape), 3,
                           workloads.SIGMA_FD8)
    y0 = np.random.default_rng(nz * ny * nx).standard_normal((2, 4) + shape)
    plan = lib_plan(B.ACOUSTIC3D, (nx, ny, nz), SCH, H, fd_order=8, n_rhs=2,
                    c2_field=to_dev(c2), c_max=float(cs.max()))
    f0, delay, w = 20.0, 0.05, 40.0
    plan.set_sources([0], [((nz - 1) * ny + ny - 1) * nx + nx - 1], [w], f0, delay)
    plan.set_variant(variant)
    got = plan.step(to_dev(y0), t0=0.01, n_macro=2).cpu().numpy()
    for rhs in range(2):
        srcs = [OP.Source((nz - 1, ny - 1, nx - 1), f0, delay, w)] if rhs == 0 else []
        op = OP.Acoustic(shape, c2=c2, r=4, sources=srcs)
        want = G.integrate(op, 0.01, y0[rhs], H, 2, steps, c)
        assert rel_err(got[rhs], want, 0) <= TOL64, rhs


@pytest.mark.parametrize("m,order", [(5, 4), (9, 8)])
def test_advection1d_minimum_grids_vs_oracle(m, order):
    steps, c = oracle_weights(SCH)
    sig = workloads.SIGMA_FD4 if order == 4 else workloads.SIGMA_FD8
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / m, 1, sig)
    u0 = np.random.default_rng(m).standard_normal((3, 1, m))
    plan = lib_plan(B.ADVECT1D, (m,), SCH, H, fd_order=order, n_rhs=3)
    got = plan.step(to_dev(u0), n_macro=5).cpu().numpy()
    for rhs in range(3):
        want = G.integrate(OP.Advection1D(m, r=order // 2), 0.0, u0[rhs], H, 5, steps, c)
        assert rel_err(got[rhs], want, 0) <= TOL64, rhs


@pytest.mark.parametrize("m", [4, 5])
def test_fourier_derivative_minimum_grids_vs_oracle(m):
    sch = schemes.GBS_8_6
    steps, c = oracle_weights(sch)
    H = 0.02 / m
    u0 = np.random.default_rng(40 + m).standard_normal((1, 1, m))
    plan = lib_plan(B.ADVECT1D, (m,), sch, H, fd_order=B.FD_SPECTRAL)
    got = plan.step(to_dev(u0), n_macro=4).cpu().numpy()
    want = G.integrate(OP.SpectralAdvection1D(m), 0.0, u0[0], H, 4, steps, c)
    assert rel_err(got[0], want, 0) <= TOL64


def test_batch_of_minimum_and_one_sided_grids_vs_oracle():
    # instances at the stencil's smallest size next to ordinary ones, in the
    # shared launches of one batch
    steps, c = oracle_weights(SCH)
    _, w, _ = scheme_weights(SCH)
    sizes = [(5, 5), (131, 5), (5, 131), (64, 64), (6, 7)]   # (nx, ny)
    inst, y0 = [], []
    rng = np.random.default_rng(77)
    for i, (nx, ny) in enumerate(sizes):
        cs = fields.lognormal_speed((ny, nx), seed=200 + i)
        H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                               workloads.SIGMA_FD4)
        inst.append(dict(n=(nx, ny), H=H, c2_field=to_dev(cs ** 2), c_max=float(cs.max()),
                         c2np=cs ** 2))
        y0.append(rng.standard_normal((3, ny, nx)))
    for variant, band in ((B.VARIANT_TEMPORAL_S5, 0), (B.VARIANT_TEMPORAL, 3),
                          (B.VARIANT_TEMPORAL_WG8, 64)):
        batch = GBSBatch(inst, 8, steps, w)
        batch.set_variant(variant, band)
        ys = [to_dev(a[None]) for a in y0]
        batch.step(ys, n_macro=2)
        for y, a, it in zip(ys, y0, inst):
            nx, ny = it["n"]
            op = OP.Acoustic((ny, nx), c2=it["c2np"], r=2)
            want = G.integrate(op, 0.0, a, it["H"], 2, steps, c)
            assert rel_err(y.cpu().numpy()[0], want, 0) <= TOL64, (variant, it["n"])


@pytest.mark.parametrize("variant", [B.VARIANT_FLAT, B.VARIANT_TEMPORAL])
@pytest.mark.parametrize("shape", [(5, 5), (5, 131), (131, 5)], ids=["5x5", "5x131", "131x5"])
def test_adjoint_minimum_grids_vs_oracle(shape, variant):
    # the streaming and the blocked adjoint (levels regenerated by reversal)
    # of one macro step, with a c^2 gradient and a source
    ny, nx = shape
    steps, c = oracle_weights(SCH)
    c2, cmax, H, src = _acoustic2d(shape, 2, seed=3 * ny + nx)
    plan = lib_plan(B.ACOUSTIC2D, (nx, ny), SCH, H, c2_field=to_dev(c2), c_max=cmax)
    (iy, ix) = src["idx"]
    plan.set_sources([0], [iy * nx + ix], [src["w"]], src["f0"], src["delay"])
    plan.set_variant(variant)
    rng = np.random.default_rng(nx * ny)
    y0 = rng.standard_normal((3, ny, nx))
    wbar = rng.standard_normal((3, ny, nx))
    t0 = 0.6 * src["delay"]
    ybar = to_dev(wbar[None])
    grad = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    plan.adjoint_step(t0, to_dev(y0[None]), ybar, grad_c2=grad)
    op = OP.Acoustic((ny, nx), c2=c2, r=2,
                     sources=[OP.Source(src["idx"], src["f0"], src["delay"], src["w"])])
    want_y, want_g = AD.macro_step_adjoint(op, t0, y0, H, steps, c, wbar)
    assert rel_err(ybar.cpu().numpy()[0], want_y, 0) <= TOL64
    assert rel_err(grad.cpu().numpy(), want_g, None) <= TOL64


def test_adjoint_3d_minimum_grid_vs_oracle():
    shape = (9, 9, 9)
    steps, c = oracle_weights(SCH)
    cs = fields.lognormal_speed(shape, seed=19)
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / 9, 3, workloads.SIGMA_FD8)
    plan = lib_plan(B.ACOUSTIC3D, (9, 9, 9), SCH, H, fd_order=8, c2_field=to_dev(c2),
                    c_max=float(cs.max()))
    rng = np.random.default_rng(23)
    y0 = rng.standard_normal((4,) + shape)
    wbar = rng.standard_normal((4,) + shape)
    for variant in (B.VARIANT_FLAT, B.VARIANT_MARCH8, B.VARIANT_TILE3D):
        plan.set_variant(variant)
        ybar = to_dev(wbar[None])
        grad = torch.zeros(shape, dtype=torch.float64, device="cuda")
        plan.adjoint_step(0.0, to_dev(y0[None]), ybar, grad_c2=grad)
        want_y, want_g = AD.macro_step_adjoint(OP.Acoustic(shape, c2=c2, r=4), 0.0, y0, H,
                                               steps, c, wbar)
        assert rel_err(ybar.cpu().numpy()[0], want_y, 0) <= TOL64, variant
        assert rel_err(grad.cpu().numpy(), want_g, None) <= TOL64, variant


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_zero_state_stays_exactly_zero(dtype):
    # f is linear in y with no source: every level, average and combination
    # of the zero state is +0 or -0, for every variant
    for op, n, order, variants in (
            (B.ACOUSTIC2D, (131, 70), 4, VARIANTS_FD4),
            (B.ACOUSTIC3D, (70, 9, 33), 8, VARIANTS_3D)):
        shape = tuple(reversed(n))
        cs = fields.lognormal_speed(shape, seed=5)
        d = len(n)
        sig = workloads.SIGMA_FD4 if order == 4 else workloads.SIGMA_FD8
        H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(n), d, sig)
        for v in variants:
            plan = lib_plan(op, n, SCH, H, fd_order=order, dtype=dtype,
                            c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()))
            plan.set_variant(v)
            y = torch.zeros((1, d + 1) + shape, dtype=dtype, device="cuda")
            out = plan.step(y, n_macro=3)
            assert int(torch.count_nonzero(out)) == 0, (op, v)
