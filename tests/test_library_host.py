"""CPU-side checks of the C-ABI library: it loads, exports what the header
declares, and its host-only logic (exact weights, ISB, plan validation)
agrees with the oracle.  No kernel is launched."""
import ctypes
from fractions import Fraction

import pytest

from oracle import stability as S
from oracle import weights as W
from paper_1907_11771_amd import binding as B
from synth import schemes, workloads


def test_library_exports_every_header_symbol():
    L = B.lib()
    names = B.header_symbols()
    assert "gbs_step" in names and "gbs_weights" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("sch", schemes.ALL, ids=lambda s: s["name"])
def test_weights_match_oracle_exactly(sch):
    pairs = [tuple(int(v) for v in x.split("/")) for x in sch["c_free"]]
    w, isb = B.weights(sch["p"], sch["steps"], sch["free_idx"], pairs)
    exact = W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    assert w == W.to_fp64(exact)                     # bit-identical nearest doubles
    want = S.isb(S.extrapolated_poly(sch["steps"], exact))
    # located in long double with a rounding-bound threshold: ~1e-7 relative
    assert isb == pytest.approx(want, rel=1e-6, abs=1e-12)


def test_isb_of_fp64_weights_and_zero_case():
    # order 6: no coverage for the exact weights; rounding the weights to
    # FP64 leaves an O(eps) low-order term, so the rounded polynomial covers
    # at most a sliver of the axis
    assert B.weights(6, [2, 4, 6])[1] == 0.0
    w = W.to_fp64(W.weights(6, [2, 4, 6]))
    assert B.isb([2, 4, 6], w) < 0.2
    w = W.to_fp64(W.weights(4, [2, 4]))
    assert B.isb([2, 4], w) == pytest.approx(3.3635857, abs=1e-6)


@pytest.mark.parametrize("steps,err", [([2, 3], B.GBS_ESTEPS), ([2, 2], B.GBS_ESTEPS),
                                       ([0, 2], B.GBS_ESTEPS)])
def test_weights_reject_bad_steps(steps, err):
    with pytest.raises(B.GBSError) as e:
        B.weights(4, steps)
    assert e.value.status == err


def test_weights_reject_bad_order():
    with pytest.raises(B.GBSError) as e:
        B.weights(5, [2, 4, 6])
    assert e.value.status == B.GBS_EORDER
    with pytest.raises(B.GBSError) as e:
        B.weights(8, [2, 4, 6])                          # k < p/2
    assert e.value.status == B.GBS_ESTEPS


# plan validation runs entirely on the host: a dummy (never dereferenced)
# workspace address stands in for device memory, and no step is taken.
FAKE_WS = 1 << 20


def _plan(op, n, p, steps, w, H, **kw):
    pr = B.make_problem(op, n, **kw)
    sc = B.make_scheme(p, steps, w)
    nb = B.workspace_bytes(pr, sc)
    h = B.plan_create(pr, sc, H, FAKE_WS, nb)
    B.plan_destroy(h)
    return nb


def _cfg2():
    sch = schemes.ORDER8_K6
    pairs = [tuple(int(v) for v in x.split("/")) for x in sch["c_free"]]
    w, _ = B.weights(8, sch["steps"], sch["free_idx"], pairs)
    return list(sch["steps"]), w


def test_workspace_bytes_formula():
    steps, w = _cfg2()
    nb = _plan(B.ACOUSTIC2D, (64, 32), 8, steps, w, 1e-3)
    pts = 64 * 32 * 3
    assert nb == 512 + 16384 + pts * 8 + 4 * 6 * pts * 8   # sources, receivers, acc, pairs


def test_plan_stability_limit_is_sharp():
    steps, w = _cfg2()
    n = 256
    lim = workloads.stable_H(workloads.ISB_ORDER8_K6, 1.0, 1.0 / n, 2, workloads.SIGMA_FD4, 1.0)
    _plan(B.ACOUSTIC2D, (n, n), 8, steps, w, 0.999 * lim)
    with pytest.raises(B.GBSError) as e:
        _plan(B.ACOUSTIC2D, (n, n), 8, steps, w, 1.002 * lim)
    assert e.value.status == B.GBS_EUNSTABLE
    # flag turns the check off
    _plan(B.ACOUSTIC2D, (n, n), 8, steps, w, 2 * lim, flags=B.FLAG_NO_STABILITY_CHECK)


def test_plan_rejects_order_2_mod_4_and_bad_weights():
    w6 = W.to_fp64(W.weights(6, [2, 4, 6]))
    with pytest.raises(B.GBSError) as e:
        _plan(B.ADVECT1D, (64,), 6, [2, 4, 6], w6, 1e-3)
    assert e.value.status == B.GBS_EORDER
    steps, w = _cfg2()
    bad = list(w)
    bad[0] += 1e-6
    with pytest.raises(B.GBSError) as e:
        _plan(B.ACOUSTIC2D, (64, 64), 8, steps, bad, 1e-4)
    assert e.value.status == B.GBS_EORDER


@pytest.mark.parametrize("kw", [dict(n=(4, 64)), dict(n=(64, 8), fd_order=8),
                                dict(n=(64, 64), fd_order=6),
                                dict(n=(64, 64), n_rhs=0), dict(n=(64, 64), dtype=7),
                                dict(n=(64, 64), c2=-1.0)])
def test_plan_rejects_bad_problem(kw):
    steps, w = _cfg2()
    n = kw.pop("n")
    with pytest.raises(B.GBSError) as e:
        _plan(B.ACOUSTIC2D, n, 8, steps, w, 1e-5, **kw)
    assert e.value.status in (B.GBS_EINVAL, B.GBS_EUNSUPPORTED)


def test_plan_rejects_small_or_misaligned_workspace():
    steps, w = _cfg2()
    pr = B.make_problem(B.ACOUSTIC2D, (64, 64))
    sc = B.make_scheme(8, steps, w)
    nb = B.workspace_bytes(pr, sc)
    with pytest.raises(B.GBSError) as e:
        B.plan_create(pr, sc, 1e-4, FAKE_WS, nb - 1)
    assert e.value.status == B.GBS_ENOMEM
    with pytest.raises(B.GBSError) as e:
        B.plan_create(pr, sc, 1e-4, FAKE_WS + 8, nb)
    assert e.value.status == B.GBS_EINVAL


def test_algorithmic_bytes_of_both_schedules():
    steps, w = _cfg2()
    pr = B.make_problem(B.ACOUSTIC2D, (64, 32))
    sc = B.make_scheme(8, steps, w)
    nb = B.workspace_bytes(pr, sc)
    h = B.plan_create(pr, sc, 1e-4, FAKE_WS, nb)
    try:
        out = [ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()]
        v = ctypes.c_int32()
        B.check(B.lib().gbs_plan_get_variant(h, ctypes.byref(v)))
        assert v.value == B.VARIANT_TEMPORAL_S5                  # the 2-D default
        pts = 64 * 32
        # the default (at most 5 evaluations per pass): N = 2, 4 take one pass
        # (write y*), N = 6, 8 two, N = 10, 12 three (2 levels between
        # passes); round 0 reads y0 once; a combine kernel
        B.check(B.lib().gbs_plan_algorithmic_bytes(h, *[ctypes.byref(x) for x in out]))
        assert out[0].value == pts * (24 + 2 * 24 + 2 * (48 + 48 + 24) + 2 * (48 + 96 + 72))
        assert out[1].value == 3
        assert out[2].value == pts * (6 * 24 + 24) and out[3].value == 1
        # f(t0, y0) shared and the combination fused: N = 2, 4 one pass, N = 6,
        # 8, 10 two, N = 12 three, alone in round 3, where it also forms
        # y_out from the other five y*; round 0 reads y0 and F_0 once
        B.check(B.lib().gbs_plan_set_form(h, B.FORM_SHARED_F0 | B.FORM_FUSED_COMBINE))
        B.check(B.lib().gbs_plan_algorithmic_bytes(h, *[ctypes.byref(x) for x in out]))
        assert out[0].value == pts * (48 + 2 * 24 + 3 * (48 + 48 + 24)
                                      + (48 + 48 + 48 + 48 + 5 * 24 + 24))
        assert out[1].value == 3
        assert out[2].value == pts * 48 and out[3].value == 1  # f(t0, y0): y0 in, F_0 out
        B.check(B.lib().gbs_plan_set_form(h, 0))
        # at most 7 evaluations per pass: N = 2, 4, 6 one pass, N = 8, 10, 12
        # two; y0, which the six first passes share, counts once
        B.check(B.lib().gbs_plan_set_variant(h, B.VARIANT_TEMPORAL))
        B.check(B.lib().gbs_plan_algorithmic_bytes(h, *[ctypes.byref(x) for x in out]))
        assert out[0].value == pts * (24 + 3 * 24 + 3 * (48 + 48 + 24))
        assert out[1].value == 2
        assert out[2].value == pts * (6 * 24 + 24) and out[3].value == 1
        B.check(B.lib().gbs_plan_set_variant(h, B.VARIANT_FLAT))
        B.check(B.lib().gbs_plan_algorithmic_bytes(h, *[ctypes.byref(x) for x in out]))
        # streaming: 72 B per stored leap-frog level, last steps 48 B + accumulator
        want = sum((n - 1) * 72 for n in steps) + 48 * 6 + 24 + 4 * 48 + 48
        assert out[0].value == pts * want and out[1].value == 12
        assert out[2].value == pts * 7 * 24                     # first evaluation
    finally:
        B.plan_destroy(h)


def test_batch_plan_validation_on_host():
    steps, w = _cfg2()
    sc = B.make_scheme(8, steps, w)
    probs = (B.Problem * 3)()
    for i, n in enumerate([(64, 64), (100, 72), (33, 40)]):
        probs[i] = B.make_problem(B.ACOUSTIC2D, n)
    Hs = (ctypes.c_double * 3)(1e-4, 1e-4, 1e-4)
    nb = ctypes.c_size_t()
    B.check(B.lib().gbs_batch_workspace_bytes(3, probs, ctypes.byref(sc), ctypes.byref(nb)))
    h = ctypes.c_void_p()
    B.check(B.lib().gbs_batch_plan_create(ctypes.byref(h), 3, probs, ctypes.byref(sc), Hs,
                                          FAKE_WS, nb.value, None))
    upd = ctypes.c_double()
    B.check(B.lib().gbs_batch_updates_per_macro_step(h, ctypes.byref(upd)))
    assert upd.value == (64 * 64 + 100 * 72 + 33 * 40) * 43
    B.check(B.lib().gbs_batch_plan_destroy(h))
    # one unstable instance rejects the batch
    Hs[1] = 1.0
    st = B.lib().gbs_batch_plan_create(ctypes.byref(h), 3, probs, ctypes.byref(sc), Hs,
                                       FAKE_WS, nb.value, None)
    assert st == B.GBS_EUNSTABLE
    # 3-D instances are not batched
    probs[2] = B.make_problem(B.ACOUSTIC3D, (16, 16, 16))
    Hs[1] = 1e-4
    st = B.lib().gbs_batch_plan_create(ctypes.byref(h), 3, probs, ctypes.byref(sc), Hs,
                                       FAKE_WS, 1 << 40, None)
    assert st == B.GBS_EUNSUPPORTED


def test_3d_variants_on_host():
    steps, w = _cfg2()
    pr = B.make_problem(B.ACOUSTIC3D, (16, 12, 10), fd_order=8)
    sc = B.make_scheme(8, steps, w)
    nb = B.workspace_bytes(pr, sc)
    h = B.plan_create(pr, sc, 1e-4, FAKE_WS, nb)
    try:
        v = ctypes.c_int32()
        B.check(B.lib().gbs_plan_get_variant(h, ctypes.byref(v)))
        assert v.value == B.VARIANT_TILE3D                      # LDS-tiled by default
        for ok in (B.VARIANT_FLAT, B.VARIANT_MARCH8, B.VARIANT_MARCH16, B.VARIANT_PLAIN,
                   B.VARIANT_TILE3D):
            B.check(B.lib().gbs_plan_set_variant(h, ok))
        for bad in (B.VARIANT_MARCH8_NT, B.VARIANT_TEMPORAL, B.VARIANT_TEMPORAL_WG4):
            assert B.lib().gbs_plan_set_variant(h, bad) == B.GBS_EUNSUPPORTED
    finally:
        B.plan_destroy(h)
    pr = B.make_problem(B.ACOUSTIC2D, (64, 64))
    h = B.plan_create(pr, sc, 1e-4, FAKE_WS, B.workspace_bytes(pr, sc))
    try:
        assert B.lib().gbs_plan_set_variant(h, B.VARIANT_TILE3D) == B.GBS_EUNSUPPORTED
        assert B.lib().gbs_plan_set_variant(h, 14) == B.GBS_EINVAL
    finally:
        B.plan_destroy(h)


def test_stability_check_uses_the_exact_scheme_behind_rounded_weights():
    # the fully determined order-8 scheme {2,16,18,20}: its FP64 weights sum
    # to more than 1 by rounding (taken literally, ISB 0); the plan checks
    # the exact scheme (ISB 12.177) and still rejects H beyond it
    steps = [2, 16, 18, 20]
    w, isb = B.weights(8, steps)
    assert isb == pytest.approx(12.177232, abs=1e-5)
    assert B.isb(steps, w) < 1.0
    pr = B.make_problem(B.ACOUSTIC2D, (64, 64))
    sc = B.make_scheme(8, steps, w)
    nb = B.workspace_bytes(pr, sc)
    rho = 1.3722220 * (64 ** 2 * 2) ** 0.5
    h = B.plan_create(pr, sc, 0.99 * isb / rho, FAKE_WS, nb)
    B.plan_destroy(h)
    with pytest.raises(B.GBSError) as ei:
        B.plan_create(pr, sc, 1.01 * isb / rho, FAKE_WS, nb)
    assert ei.value.status == B.GBS_EUNSTABLE


def test_lanes_validation_on_host():
    steps, w = _cfg2()
    pr = B.make_problem(B.ACOUSTIC2D, (64, 32))
    sc = B.make_scheme(8, steps, w)
    h = B.plan_create(pr, sc, 1e-4, FAKE_WS, B.workspace_bytes(pr, sc))
    try:
        for bad in (0, 5, -1):
            assert B.lib().gbs_plan_set_lanes(h, bad) == B.GBS_EINVAL
        B.check(B.lib().gbs_plan_set_lanes(h, 1))
    finally:
        B.plan_destroy(h)


def test_rk4_entry_validates_on_host():
    # every check of gbs_rk4_step runs before any device call: RK4's
    # imaginary stability boundary 2 sqrt 2 (App. A) against h rho
    steps, w = _cfg2()
    n = 64
    pr = B.make_problem(B.ACOUSTIC2D, (n, n))
    sc = B.make_scheme(8, steps, w)
    h = B.plan_create(pr, sc, 1e-4, FAKE_WS, B.workspace_bytes(pr, sc))
    rho = 1.3722220 * (2 * n * n) ** 0.5
    lim = 2 * 2 ** 0.5 / rho
    ptr = ctypes.c_void_p(FAKE_WS)
    try:
        L = B.lib()
        assert L.gbs_rk4_step(h, 0.0, 1, 1.001 * lim, ptr, ptr) == B.GBS_EUNSTABLE
        assert L.gbs_rk4_step(h, 0.0, -1, 0.5 * lim, ptr, ptr) == B.GBS_EINVAL
        assert L.gbs_rk4_step(h, 0.0, 1, 0.0, ptr, ptr) == B.GBS_EINVAL
        assert L.gbs_rk4_step(h, float("nan"), 1, 0.5 * lim, ptr, ptr) == B.GBS_EINVAL
        assert L.gbs_rk4_step(h, 0.0, 1, 0.5 * lim, None, ptr) == B.GBS_EINVAL
        assert L.gbs_rk4_step(None, 0.0, 1, 0.5 * lim, ptr, ptr) == B.GBS_EINVAL
        # n_steps = 0 in place is a no-op that touches nothing
        assert L.gbs_rk4_step(h, 0.0, 0, 0.5 * lim, ptr, ptr) == B.GBS_OK
    finally:
        B.plan_destroy(h)


def test_fourier_derivative_plans_on_host():
    # spectral advection (Sect. 4.1): rho = pi M; ADVECT1D only; 4 <= M <= 8192
    steps, w = _cfg2()
    sc = B.make_scheme(8, steps, w)
    for op, n in ((B.ACOUSTIC2D, (32, 32)), (B.ACOUSTIC3D, (16, 16, 16))):
        with pytest.raises(B.GBSError) as ei:
            B.workspace_bytes(B.make_problem(op, n, fd_order=B.FD_SPECTRAL), sc)
        assert ei.value.status == B.GBS_EUNSUPPORTED
    for m in (3, 8193):
        with pytest.raises(B.GBSError) as ei:
            B.workspace_bytes(B.make_problem(B.ADVECT1D, (m,), fd_order=B.FD_SPECTRAL), sc)
        assert ei.value.status == B.GBS_EINVAL
    m = 100
    pr = B.make_problem(B.ADVECT1D, (m,), fd_order=B.FD_SPECTRAL)
    fd = B.make_problem(B.ADVECT1D, (m,), fd_order=4)
    nb = B.workspace_bytes(pr, sc)
    assert nb == B.workspace_bytes(fd, sc) + 512      # the 49 weights b_k (392 B), 256-aligned
    isb = B.isb(steps, w)
    lim = isb / (3.141592653589793 * m)
    B.plan_destroy(B.plan_create(pr, sc, 0.999 * lim, FAKE_WS, nb))
    with pytest.raises(B.GBSError) as ei:
        B.plan_create(pr, sc, 1.001 * lim, FAKE_WS, nb)
    assert ei.value.status == B.GBS_EUNSTABLE
    h = B.plan_create(pr, sc, 0.5 * lim, FAKE_WS, nb)
    ptr = ctypes.c_void_p(FAKE_WS)
    try:
        rk_lim = 2 * 2 ** 0.5 / (3.141592653589793 * m)
        assert B.lib().gbs_rk4_step(h, 0.0, 1, 1.001 * rk_lim, ptr, ptr) == B.GBS_EUNSTABLE
    finally:
        B.plan_destroy(h)


def test_kept_pairs_validation_on_host():
    # every rejection happens before any device call
    steps, w = _cfg2()
    sc = B.make_scheme(8, steps, w)
    ptr = ctypes.c_void_p(FAKE_WS)
    L = B.lib()
    for fd, variant, want in ((8, 0, B.GBS_EUNSUPPORTED), (4, B.VARIANT_FLAT, B.GBS_EUNSUPPORTED)):
        pr = B.make_problem(B.ACOUSTIC2D, (64, 32), fd_order=fd)
        h = B.plan_create(pr, sc, 1e-4, FAKE_WS, B.workspace_bytes(pr, sc))
        try:
            if variant:
                B.check(L.gbs_plan_set_variant(h, variant))
            assert L.gbs_step_keep_pairs(h, 0.0, 1, ptr, ptr, ptr) == want
            assert L.gbs_adjoint_step_pairs(h, 0.0, ptr, ptr, ptr, None, None, ptr,
                                            1 << 40) == want
        finally:
            B.plan_destroy(h)
    pr = B.make_problem(B.ACOUSTIC2D, (64, 32))
    h = B.plan_create(pr, sc, 1e-4, FAKE_WS, B.workspace_bytes(pr, sc))
    try:
        assert L.gbs_step_keep_pairs(h, 0.0, 1, ptr, ptr, None) == B.GBS_EINVAL
        assert L.gbs_step_keep_pairs(h, 0.0, 0, ptr, ptr, ptr) == B.GBS_EINVAL
        assert L.gbs_adjoint_step_pairs(h, 0.0, ptr, None, ptr, None, None, ptr,
                                        1 << 40) == B.GBS_EINVAL
    finally:
        B.plan_destroy(h)
