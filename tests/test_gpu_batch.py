"""GPU batching: instances of uneven size advanced together must equal the
same instances advanced one by one (bitwise: same kernels, same arithmetic),
and the oracle; the captured graph must equal eager launches on every
replay; and the batch workload at its full size (64 instances, 256^2 to
1024^2, autotuned and graph-captured as the benchmark runs it) against the
oracle, whole or on periodic windows around sampled points."""
import numpy as np
import pytest
import torch

from oracle import gbs as G
from oracle import operators as OP
from paper_1907_11771_amd import binding as B
from paper_1907_11771_amd.plan import GBSBatch, GBSPlan, scheme_weights
from synth import fields, schemes, workloads
from tests.gpu_util import oracle_weights, rel_err, to_dev

pytestmark = pytest.mark.gpu

SIZES = [(64, 64), (100, 72), (33, 40), (128, 96), (64, 200)]


def _instances(dtype):
    out = []
    for i, (nx, ny) in enumerate(SIZES):
        cs = fields.lognormal_speed((ny, nx), seed=100 + i)
        H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / max(nx, ny), 2,
                               workloads.SIGMA_FD4)
        out.append(dict(n=(nx, ny), H=H, c2_field=to_dev(cs ** 2, dtype), c_max=float(cs.max()),
                        c2np=cs ** 2))
    return out


def _states(dtype, seed=0):
    rng = np.random.default_rng(seed)
    return [to_dev(rng.standard_normal((1, 3, ny, nx)), dtype) for nx, ny in SIZES]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("variant,band", [(B.VARIANT_TEMPORAL, 64), (B.VARIANT_TEMPORAL4, 30),
                                          (B.VARIANT_TEMPORAL_S5, 128), (B.VARIANT_TEMPORAL_WG4, 64),
                                          (B.VARIANT_TEMPORAL_WG8, 48), (B.VARIANT_TEMPORAL_S6, 96)])
def test_batch_equals_single_instances(dtype, variant, band):
    sch = schemes.ORDER8_K6
    steps, w, _ = scheme_weights(sch)
    inst = _instances(dtype)
    batch = GBSBatch(inst, 8, steps, w, dtype=dtype)
    batch.set_variant(variant, band)
    ys = _states(dtype)
    ref = [y.clone() for y in ys]
    batch.step(ys, n_macro=3)
    for y, r, it in zip(ys, ref, inst):
        single = GBSPlan(B.ACOUSTIC2D, it["n"], 8, steps, w, it["H"], dtype=dtype,
                         c2_field=it["c2_field"], c_max=it["c_max"])
        single.set_variant(variant)
        B.check(B.lib().gbs_plan_set_band(single.handle, band))
        assert torch.equal(single.step(r, n_macro=3), y)


def test_batch_matches_oracle():
    sch = schemes.ORDER8_K6
    steps, c = oracle_weights(sch)
    _, w, _ = scheme_weights(sch)
    inst = _instances(torch.float64)
    batch = GBSBatch(inst, 8, steps, w)
    ys = _states(torch.float64, seed=5)
    y0 = [y.cpu().numpy()[0] for y in ys]
    batch.step(ys, n_macro=2)
    for y, a, it in zip(ys, y0, inst):
        nx, ny = it["n"]
        want = G.integrate(OP.Acoustic((ny, nx), c2=it["c2np"], r=2), 0.0, a, it["H"], 2, steps, c)
        assert rel_err(y.cpu().numpy()[0], want, 0) <= 1e-12


def test_batch_graph_replays_equal_eager():
    sch = schemes.ORDER8_K6
    steps, w, _ = scheme_weights(sch)
    inst = _instances(torch.float64)
    eager = GBSBatch(inst, 8, steps, w)
    graph = GBSBatch(inst, 8, steps, w)
    graph.set_graph(True)
    ya = _states(torch.float64, seed=9)
    yb = [y.clone() for y in ya]
    for rep in range(4):
        eager.step(ya, n_macro=2)
        graph.step(yb, n_macro=2)
        torch.cuda.synchronize()
        # unrelated eager work between the replays
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        junk.mul_(2.0).sum().item()
        for a, b in zip(ya, yb):
            assert torch.equal(a, b), rep


def test_batch_autotune_picks_a_candidate():
    sch = schemes.ORDER8_K6
    steps, w, _ = scheme_weights(sch)
    inst = _instances(torch.float64)
    batch = GBSBatch(inst, 8, steps, w)
    v, band = batch.autotune(_states(torch.float64), macro_steps=1)
    assert v in (B.VARIANT_TEMPORAL, B.VARIANT_TEMPORAL4, B.VARIANT_TEMPORAL_S5,
                 B.VARIANT_TEMPORAL_S6, B.VARIANT_TEMPORAL_WG4, B.VARIANT_TEMPORAL_WG8)
    assert band in (32, 64, 96, 128)
    ys = _states(torch.float64, seed=3)
    ref = [y.clone() for y in ys]
    batch.step(ys, n_macro=1)
    other = GBSBatch(inst, 8, steps, w)
    other.set_variant(B.VARIANT_TEMPORAL, 64)
    other.step(ref, n_macro=1)
    for a, b in zip(ys, ref):
        assert rel_err(a.cpu().numpy(), b.cpu().numpy(), 1) <= 1e-13


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 3e-5)])
def test_full_size_batch_vs_oracle(dtype, tol):
    # the batch workload itself in the benchmark's launch configuration (64
    # instances of 256^2 .. 1024^2 with their log-normal c^2 and H,
    # autotuned variant and band, graph-captured), one macro step from random
    # states: every 256^2 instance whole against the oracle, and each larger
    # instance sampled, the oracle on two periodic windows of half-width 30
    # with the instance's spacing, exact at the 9^2 points within 4 of the
    # middle (the longest sequence's 13 evaluations reach 13 x 2 = 26 points;
    # FP32 stepping held to the bound u32 sum|c| (1 + sum N_j))
    sch = schemes.ORDER8_K6
    steps, c = oracle_weights(sch)
    _, w, _ = scheme_weights(sch)
    inst = workloads.batch_instances(workloads.CONFIG_BATCH)
    rng = np.random.default_rng(64)
    y0 = [rng.standard_normal((3, n, n)) for n, _, _ in inst]
    spec = [dict(n=(n, n), H=H, c2_field=to_dev(cs * cs, dtype), c_max=float(cs.max()))
            for n, cs, H in inst]
    batch = GBSBatch(spec, 8, steps, w, dtype=dtype)
    batch.autotune([to_dev(a[None], dtype) for a in y0], macro_steps=1)
    batch.set_graph(True)
    ys = [to_dev(a[None], dtype) for a in y0]
    batch.step(ys, n_macro=1)
    hw, k = 30, 4
    whole = 0
    for i, ((n, cs, H), a, y) in enumerate(zip(inst, y0, ys)):
        got = y[0]
        if n == 256:
            want = G.macro_step(OP.Acoustic((n, n), c2=cs * cs, r=2), 0.0, a, H, steps, c)
            e = rel_err(got.double().cpu().numpy(), want, 0)
            whole += 1
            assert e <= tol, (i, n, e)
            continue
        for ctr in (tuple(int(v) for v in rng.integers(0, n, size=2)), (1, n - 2)):
            iy, ix = [np.arange(q - hw, q + hw + 1) % n for q in ctr]
            op = OP.Acoustic((2 * hw + 1,) * 2, c2=(cs * cs)[np.ix_(iy, ix)], r=2,
                             spacing=(1.0 / n, 1.0 / n))
            want = G.macro_step(op, 0.0, a[(slice(None),) + np.ix_(iy, ix)], H, steps, c)
            want = want[:, hw - k:hw + k + 1, hw - k:hw + k + 1]
            ty, tx = [torch.from_numpy(v[hw - k:hw + k + 1]).cuda() for v in (iy, ix)]
            part = got[:, ty[:, None], tx[None, :]].double().cpu().numpy()
            e = rel_err(part, want, 0)
            assert e <= tol, (i, n, ctr, e)
    assert whole > 0
