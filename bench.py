"""Benchmark: extrapolated GBS macro steps of the 2-D acoustic workload
(2048^2 periodic grid, FP64, FD4, order-8 scheme over N = 2,4,...,12) on one
MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-adjoint]
                    [--no-batch] [--no-3d]

One "step" is one macro step: all six GBS sequences (forward Euler, N_j
leap-frog steps, averaging) and the FP64 weighted combination, i.e.
1 + sum N_j = 43 RHS evaluations per grid point.  Prints one JSON line; its
"fwd_adj" object is the metric's second half, forward + adjoint time at
fixed error against the plain form (the 1024^2 differentiation workload,
400 macro steps), with the adjoint pass kernel's roofline; "batch64" holds
the batch workload in FP64 and FP32 stepping (100 macro steps) and
"acoustic3d" the 384^3 FD8 forward with 8 right-hand sides (FP32 stepping,
FP64 and the plain FP64 form beside it, LEG_3D_MACRO_STEPS macro steps).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
STREAM_BYTES_PER_UPDATE = 72.0   # FP64 2-D acoustic leap-frog update, streaming: 3 F b
LEG_3D_MACRO_STEPS = 10    # macro steps of the default line's 3-D forward leg
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1907_11771_amd", "csrc")


def source_sha():
    """Fingerprint of the library's device and launch code (every file under
    csrc/): a counter profile applies only to the code it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of ``kernel`` on ``workload`` from the counter
    summaries under profiles/ (lines "TRAFFIC {json}" written by
    --summarize-counters), or None when no summary was taken on the current
    sources for exactly that kernel and workload."""
    sha = source_sha()
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".txt"):
            continue
        with open(os.path.join(PROFILES, name)) as fh:
            for ln in fh:
                if not ln.startswith("TRAFFIC "):
                    continue
                rec = json.loads(ln[len("TRAFFIC "):])
                if (rec.get("kernel") == kernel and rec.get("workload") == workload
                        and rec.get("source_sha") == sha):
                    rec["profile"] = "profiles/" + name
                    return rec
    return None


def kernel_base_name(k):
    """'void gbs::pass2d<double, 4, 5, ...>(gbs::PassArgs<double>)' ->
    'gbs::pass2d<double, 4, 5, ...>' (the profiler's name without the return
    type and the parameter list)."""
    k = k.strip()
    if k.startswith("void "):
        k = k[5:]
    depth = 0
    for i, ch in enumerate(k):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return k[:i].strip()
    return k


def _counter_rows(path):
    """(kernel name, dispatch id, counter, value) rows of a rocprofv3
    counter_collection CSV."""
    import csv
    rows = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Kernel_Name"], int(r["Dispatch_Id"]), r["Counter_Name"],
                         float(r["Counter_Value"])))
    return rows


def summarize_counters(args):
    """Turns two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) of a kernel and the same two counters on the plain 1 GiB copy
    (--copy-calibration) into HBM bytes per launch, scaled so that the copy
    reads and writes exactly 1 GiB; prints the TRAFFIC line a profile
    summary carries (bench.py's roofline 'traffic' reads it back)."""
    fetch, write, cfetch, cwrite = args.summarize_counters

    def per_dispatch(path, counter, match):
        vals = {}
        for k, d, c, v in _counter_rows(path):
            if c == counter and match(k):
                vals[d] = vals.get(d, 0.0) + v
        return [vals[d] for d in sorted(vals)]

    is_kernel = lambda k: kernel_base_name(k) == args.kernel
    is_copy = lambda k: "copy" in k.lower() or "elementwise" in k.lower()
    f = per_dispatch(fetch, "FETCH_SIZE", is_kernel)
    w = per_dispatch(write, "WRITE_SIZE", is_kernel)
    if args.last:
        # the timed region's launches only (the autotuner's trial launches
        # of the same kernel come first)
        f, w = f[-args.last:], w[-args.last:]
    cf = per_dispatch(cfetch, "FETCH_SIZE", is_copy)
    cw = per_dispatch(cwrite, "WRITE_SIZE", is_copy)
    if not (f and w and cf and cw):
        raise SystemExit("no dispatches of %r (or of the copy) in the counter files" % args.kernel)
    gib = float(1 << 30)
    sf = gib / (max(cf) * 1024.0)      # bytes per counted KiB, from the copy
    sw = gib / (max(cw) * 1024.0)
    fb = sum(f) / len(f) * 1024.0 * sf
    wb = sum(w) / len(w) * 1024.0 * sw
    rec = dict(kernel=args.kernel, workload=args.counters_workload, source_sha=source_sha(),
               launches=len(f), fetch_scale=sf, write_scale=sw,
               fetch_bytes_per_launch=fb, write_bytes_per_launch=wb,
               bytes_per_launch=fb + wb,
               fetch_bytes_by_launch=[x * 1024.0 * sf for x in f],
               write_bytes_by_launch=[x * 1024.0 * sw for x in w])
    print("TRAFFIC " + json.dumps(rec))


def kernel_names(variant, B):
    step = {B.VARIANT_TEMPORAL: "gbs::pass2d<double, 4, 7, false, 1, false, false, false>",
            B.VARIANT_TEMPORAL4: "gbs::pass2d<double, 4, 4, false, 1, false, false, false>",
            B.VARIANT_TEMPORAL_S5: "gbs::pass2d<double, 4, 5, true, 1, false, false, false>",
            B.VARIANT_TEMPORAL_S6: "gbs::pass2d<double, 4, 6, true, 1, false, false, false>",
            B.VARIANT_TEMPORAL_WG4: "gbs::pass2d<double, 4, 7, false, 4, false, false, false>",
            B.VARIANT_TEMPORAL_WG8: "gbs::pass2d<double, 4, 7, false, 8, false, false, false>",
            B.VARIANT_FLAT: "gbs::lf_kernel<double, 4, 2>"}.get(variant,
                                                              "gbs::lf_march2d<double, 4, ...>")
    temporal = variant in (B.VARIANT_TEMPORAL, B.VARIANT_TEMPORAL4, B.VARIANT_TEMPORAL_S5,
                           B.VARIANT_TEMPORAL_S6, B.VARIANT_TEMPORAL_WG4, B.VARIANT_TEMPORAL_WG8)
    aux = "gbs::combine_kernel<double>" if temporal else "gbs::first_kernel<double, 4, 2>"
    return step, aux


def cpu_baseline(cfg, y0):
    """The oracle (NumPy FP64, one thread) on three macro steps of the same
    grid (about 15 s), as a rate per macro step."""
    from fractions import Fraction
    from oracle import gbs as G
    from oracle import operators as OP
    from oracle import weights as W
    sch = cfg["scheme"]
    exact = W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    steps, c = list(sch["steps"]), W.to_fp64(exact)
    op = OP.Acoustic((cfg["n"], cfg["n"]), c2=cfg["c2"], r=cfg["r"])
    n_cpu = 3
    t = time.perf_counter()
    G.integrate(op, 0.0, y0, cfg["H"], n_cpu, steps, c)
    dt = time.perf_counter() - t
    updates = cfg["n"] * cfg["n"] * (1 + sum(steps))
    out = dict(value=n_cpu * updates / dt, unit="grid-pt RHS updates/s", cores=1, kind="oracle",
               sample="%d macro steps of the same 2048^2 FP64 workload (43 RHS sweeps each), "
                      "%.1f s, NumPy single thread" % (n_cpu, dt))
    out["folded"] = cpu_folded(cfg, updates)
    return out


def _folded_group(args):
    """One process of the paper's CPU scheme: its sequences of one macro step
    of the oracle, on the same synthetic state (regenerated from its seed);
    returns the seconds of compute (the group's sum c_j y*_j stays local)."""
    cfg, group = args
    import numpy as np
    from oracle import gbs as G
    from oracle import operators as OP
    from synth import fields
    y0 = fields.acoustic2d_pulse_modes(cfg["n"])
    op = OP.Acoustic((cfg["n"], cfg["n"]), c2=cfg["c2"], r=cfg["r"])
    t = time.perf_counter()
    f0 = op(0.0, y0)
    part = None
    for n, cj in group:
        term = cj * G.sequence(op, 0.0, y0, f0, cfg["H"] / n, n)
        part = term if part is None else part + term
    return time.perf_counter() - t


def cpu_folded(cfg, updates):
    """The paper's own CPU scheme (Sect. 3.6) as a second reference: the
    sequences folded in pairs whose step counts add up to N_max, one process
    per group ({12}, {10, 2}, {8, 4}, {6}), each evaluating f(t0, y0) itself;
    the time of one macro step is the slowest group's.  Processes are started
    with the spawn method (fresh interpreters that touch no device)."""
    import multiprocessing as mp
    from fractions import Fraction
    from oracle import weights as W
    sch = cfg["scheme"]
    exact = W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    pairs = dict(zip(sch["steps"], W.to_fp64(exact)))
    ns = sorted(pairs)
    groups, lo, hi = [], 0, len(ns) - 1
    while lo <= hi:
        g = [ns[hi]] if lo == hi or ns[hi] == max(ns) else [ns[hi], ns[lo]]
        if len(g) == 2:
            lo += 1
        hi -= 1
        groups.append([(n, pairs[n]) for n in g])
    try:
        with mp.get_context("spawn").Pool(len(groups)) as pool:
            res = pool.map_async(_folded_group, [(cfg, g) for g in groups]).get(timeout=300)
    except Exception as e:                            # report, never hang the bench
        return dict(error="folded CPU reference failed: %r" % (e,))
    dt = max(res)
    return dict(value=updates / dt, unit="grid-pt RHS updates/s", cores=len(groups),
                kind="oracle, folded sequences",
                sample="the same macro step, groups %s, one process each, %.2f s (slowest group)"
                       % ([[n for n, _ in g] for g in groups], dt))


def batch_inputs():
    """The 64 instances (size, speed field, H) and their initial states:
    smooth ones (the 2-D workload's construction: a Gaussian pulse plus 32
    plane waves up to wavenumber 16, seed per instance), so that the FP32
    error is stated on representative data."""
    from synth import fields, workloads
    inst = workloads.batch_instances(workloads.CONFIG_BATCH)
    y0 = [fields.acoustic2d_pulse_modes(n, seed=100 + i)[None] for i, (n, _, _) in enumerate(inst)]
    return inst, y0


def batch_leg(n_macro, warmup, dtype_name, plain=True, inputs=None, pin=None):
    """64 uneven instances advanced in one batch (graph-replayed macro steps,
    autotuned variant and band, or the (variant, band) ``pin``) for
    ``n_macro`` timed macro steps, in FP64 or FP32 stepping (then with the
    error against the FP64 batch after the same steps), and the plain FP64
    form (one streaming launch per sequence per leap-frog step, instance by
    instance) per macro step."""
    import torch
    from paper_1907_11771_amd import binding as B
    from paper_1907_11771_amd.plan import GBSBatch, GBSPlan, scheme_weights
    from synth import workloads

    cfg = workloads.CONFIG_BATCH
    steps, w, _ = scheme_weights(cfg["scheme"])
    dev = torch.device("cuda:0")
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    inst, y0 = inputs or batch_inputs()
    spec = [dict(n=(n, n), H=H, c2_field=torch.from_numpy(c * c).to(dev), c_max=float(c.max()))
            for n, c, H in inst]
    batch = GBSBatch(spec, 8, steps, w, dtype=dtype, device=dev)
    if pin:
        variant, band = pin
        batch.set_variant(variant, band)
    else:
        tune = [torch.from_numpy(a).to(dev, dtype) for a in y0]
        variant, band = batch.autotune(tune, macro_steps=1)
        del tune
    batch.set_graph(True)
    ys = [torch.from_numpy(a).to(dev, dtype) for a in y0]
    batch.step(ys, n_macro=max(warmup, 1))
    ys = [torch.from_numpy(a).to(dev, dtype) for a in y0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    batch.step(ys, n_macro=n_macro)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    upd = batch.updates_per_macro_step() * n_macro
    del batch

    # accuracy of this run against the FP64 batch after the same steps
    err = None
    if dtype == torch.float32:
        ref = GBSBatch(spec, 8, steps, w, dtype=torch.float64, device=dev)
        ref.set_variant(variant, band)
        yr = [torch.from_numpy(a).to(dev) for a in y0]
        ref.step(yr, n_macro=n_macro)
        err = max(float((a.double() - b).abs().max() / b.abs().max()) for a, b in zip(ys, yr))
        del ref, yr

    # method bytes of one macro step (the passes and the combination of every
    # instance), as a single plan of the instance's size and the batch's
    # variant counts them
    step_bytes, pass_launches = 0.0, 0
    for n in sorted(set(n for n, _, _ in inst)):
        same = [(c, H) for m, c, H in inst if m == n]
        c, H = same[0]
        pl = GBSPlan(B.ACOUSTIC2D, (n, n), 8, steps, w, H, dtype=dtype,
                     c2_field=torch.from_numpy(c * c).to(dev), c_max=float(c.max()), device=dev)
        pl.set_variant(variant)
        sb, pass_launches, ab, _ = pl.algorithmic_bytes()
        step_bytes += len(same) * (sb + ab)
        del pl
    # measured HBM bytes of a macro step, where a counter summary of the
    # batch's pass and combination kernels was taken on the current sources
    forms = {B.VARIANT_TEMPORAL: "7, false, 1", B.VARIANT_TEMPORAL4: "4, false, 1",
             B.VARIANT_TEMPORAL_S5: "5, true, 1", B.VARIANT_TEMPORAL_S6: "6, true, 1",
             B.VARIANT_TEMPORAL_WG4: "7, false, 4", B.VARIANT_TEMPORAL_WG8: "7, false, 8"}
    tname = "double" if dtype == torch.float64 else "float"
    kpass = "gbs::pass2d_batch<%s, 4, %s>" % (tname, forms.get(variant, "?"))
    tp = measured_traffic(kpass, cfg["name"])
    tc = measured_traffic("gbs::combine_batch<%s>" % tname, cfg["name"])
    traffic_bytes = (pass_launches * tp["bytes_per_launch"] + tc["bytes_per_launch"]
                     if tp and tc else None)

    # the plain FP64 form on the same instances (a few macro steps, per macro step)
    plain_ms = None
    if plain:
        plain_steps = 3
        plain_s = 0.0
        for (n, c, H), a in zip(inst, y0):
            pl = GBSPlan(B.ACOUSTIC2D, (n, n), 8, steps, w, H, dtype=torch.float64,
                         c2_field=torch.from_numpy(c * c).to(dev), c_max=float(c.max()),
                         device=dev)
            pl.set_variant(B.VARIANT_PLAIN)
            y = torch.from_numpy(a).to(dev)
            pl.step(y, y, n_macro=1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            pl.step(y, y, n_macro=plain_steps)
            torch.cuda.synchronize()
            plain_s += time.perf_counter() - t
            del pl, y
        plain_ms = plain_s * 1e3 / plain_steps
    del spec, ys
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ms = dt * 1e3 / n_macro
    return dict(
        updates_per_s=upd / dt, ms_per_step=ms, steps=n_macro, dtype=dtype_name,
        config=dict(workload=cfg["name"], instances=len(inst),
                    sizes=sorted(set(n for n, _, _ in inst)), points=sum(n * n for n, _, _ in inst),
                    evals_per_macro_step=1 + sum(steps), graph=True,
                    **{"pinned" if pin else "autotuned": dict(variant=variant, band=band)}),
        plain_fp64_ms_per_step=plain_ms,
        speedup_vs_plain_fp64=plain_ms / ms if plain_ms else None,
        max_rel_err_vs_fp64=err,
        # whole macro steps (passes and combination) against the HBM peak
        bandwidth=dict(method_bytes_per_step=step_bytes,
                       achieved=step_bytes / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                       frac=step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       pass_kernel=kpass, pass_launches_per_step=pass_launches,
                       traffic_bytes_per_step=traffic_bytes,
                       traffic=traffic_bytes / (ms * 1e-3) / 1e9 if traffic_bytes else None,
                       traffic_profile=tp["profile"] if tp and tc else None))


def bench_batch(args):
    """The batch workload on its own line (batch_leg)."""
    from synth import workloads
    if args.steps == 500:                 # the default: the batch workload's own length
        args.steps = workloads.CONFIG_BATCH["n_macro"]
    leg = batch_leg(args.steps, args.warmup, args.dtype,
                    pin=(args.variant, args.band) if args.variant else None)
    rec = dict(
        metric="grid-pt RHS updates/s", value=leg["updates_per_s"], unit="grid-pt RHS updates/s",
        n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=leg["ms_per_step"],
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype=args.dtype,
        data="synthetic", config=leg["config"],
        plain_fp64_ms_per_step=leg["plain_fp64_ms_per_step"],
        speedup_vs_plain_fp64=leg["speedup_vs_plain_fp64"],
        max_rel_err_vs_fp64=leg["max_rel_err_vs_fp64"], bandwidth=leg["bandwidth"],
    )
    print(json.dumps(rec), flush=True)


def bench_adjoint(args):
    """The forward + adjoint workload on its own line (adjoint_leg)."""
    nm = None if args.steps == 500 else args.steps
    rec = adjoint_leg(nm, args.grid or None)
    print(json.dumps(rec), flush=True)


def adjoint_leg(n_macro=None, grid=None):
    """Forward + checkpointed adjoint of the receiver misfit (gradients with
    respect to c^2 and p(0)) on the 1024^2 workload: FP64 blocked forward,
    FP32 stepping, and the plain FP64 form; the FP32 gradient's error is
    stated against the FP64 one.  Also the blocked adjoint pass kernel's
    roofline: its algorithmic bytes over its HIP-event time in one more
    FP64 backward pass on one lane."""
    import numpy as np
    import torch
    from paper_1907_11771_amd import binding as B
    from paper_1907_11771_amd.autograd import receiver_traces
    from paper_1907_11771_amd.plan import GBSPlan, scheme_weights
    from synth import fields, workloads

    cfg = workloads.CONFIG_ADJOINT
    n, nm = grid or cfg["n"], cfg["n_macro"] if n_macro is None else n_macro
    wname = cfg["name"] if n == cfg["n"] else cfg["name"].replace(str(cfg["n"]), str(n))
    steps, w, _ = scheme_weights(cfg["scheme"])
    dev = torch.device("cuda:0")
    cs = fields.lognormal_speed((n, n), seed=cfg["speed_seed"])
    c2 = cs ** 2
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, cs.max(), 1.0 / n, 2, workloads.SIGMA_FD4)
    s = fields.ricker_source_2d(n)
    rec = fields.edge_receivers_2d(n, count=cfg["receivers"])
    c2_obs = c2 * np.exp(0.1 * fields.gaussian_random_field((n, n), seed=cfg["data_seed"]))

    def make(dtype, variant=0):
        pl = GBSPlan(B.ACOUSTIC2D, (n, n), 8, steps, w, H, dtype=dtype,
                     c2_field=torch.from_numpy(c2).to(dev), c_max=float(cs.max()) * 1.01,
                     device=dev)
        if variant:
            pl.set_variant(variant)
        else:
            pl.autotune(torch.zeros(pl.state_shape, dtype=dtype, device=dev), macro_steps=3)
        pl.set_sources([0], [s["idx"][0] * n + s["idx"][1]], [s["weight"]], s["f0"], s["delay"])
        if not variant:
            pl.autotune_adjoint(torch.randn(pl.state_shape, dtype=dtype, device=dev))
        pl.set_receivers([0] * len(rec), [int(r[0]) * n + int(r[1]) for r in rec])
        return pl

    ref = make(torch.float64)
    with torch.no_grad():
        data = receiver_traces(ref, torch.zeros((1, 3, n, n), dtype=torch.float64, device=dev),
                               torch.from_numpy(c2_obs).to(dev), nm)

    def run(pl, dtype):
        y0 = torch.zeros((1, 3, n, n), dtype=dtype, device=dev, requires_grad=True)
        c2v = torch.from_numpy(c2).to(dev, dtype).requires_grad_(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        tr = receiver_traces(pl, y0, c2v, nm, checkpoint_every=cfg["checkpoint_every"])
        loss = 0.5 * ((tr.double() - data) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t, t2 - t1, c2v.grad.double(), float(loss.detach())

    def warm(pl, dtype):
        y0 = torch.zeros((1, 3, n, n), dtype=dtype, device=dev, requires_grad=True)
        c2v = torch.from_numpy(c2).to(dev, dtype).requires_grad_(True)
        tr = receiver_traces(pl, y0, c2v, 4, checkpoint_every=2)
        tr.sum().backward()
        torch.cuda.synchronize()

    forms = {"f64": (torch.float64, 0), "f32": (torch.float32, 0),
             "plain": (torch.float64, B.VARIANT_PLAIN)}
    plans = {k: make(dt, v) for k, (dt, v) in forms.items()}
    for k, (dt, _) in forms.items():
        warm(plans[k], dt)
    for k, (dt, _) in forms.items():
        run(plans[k], dt)          # full-length untimed pass: allocations settle
    f64, b64, g64, l64 = run(plans["f64"], torch.float64)
    f32, b32, g32, l32 = run(plans["f32"], torch.float32)
    fpl, bpl, gpl, _ = run(plans["plain"], torch.float64)
    tuned = {k: plans[k].variant() for k in ("f64", "f32")}
    rel = lambda a, b: float((a - b).norm() / b.norm())
    # the adjoint pass kernel alone: one more FP64 backward on one lane with
    # every pass launch bracketed by HIP events
    p64 = plans["f64"]
    lanes64 = p64.adjoint_lanes
    p64.adjoint_lanes = 1
    y0 = torch.zeros((1, 3, n, n), dtype=torch.float64, device=dev, requires_grad=True)
    c2v = torch.from_numpy(c2).to(dev).requires_grad_(True)
    tr = receiver_traces(p64, y0, c2v, nm, checkpoint_every=cfg["checkpoint_every"])
    loss = 0.5 * ((tr - data) ** 2).sum()
    torch.cuda.synchronize()
    p64.set_timing(1)
    loss.backward()
    torch.cuda.synchronize()
    adj_ms, adj_n, adj_bytes = p64.get_adjoint_timing()
    p64.set_timing(0)
    p64.adjoint_lanes = lanes64
    adj_kernel = "gbs::adj_pass2d<double, 3, true>"
    prof = measured_traffic(adj_kernel, wname)
    adj_launch_s = adj_ms * 1e-3 / max(adj_n, 1)
    achieved = adj_bytes / max(adj_n, 1) / adj_launch_s / 1e9 if adj_n else None
    upd = n * n * (1 + sum(steps)) * nm
    rec_out = dict(
        metric="fwd+adjoint time at fixed error vs plain", value=(f64 + b64), unit="s",
        higher_is_better=False, n_gpus=1, steps=nm, warmup=1, dtype="f64", data="synthetic",
        config=dict(workload=wname, grid=[n, n], macro_steps=nm,
                    checkpoint_every=cfg["checkpoint_every"], receivers=len(rec)),
        fp64=dict(forward_s=f64, adjoint_s=b64, forward_updates_per_s=upd / f64),
        fp32_stepping=dict(forward_s=f32, adjoint_s=b32,
                           grad_c2_rel_err_vs_fp64=rel(g32, g64) if g64.norm() > 0 else None,
                           misfit_rel_err_vs_fp64=abs(l32 - l64) / abs(l64) if l64 else None),
        plain_fp64=dict(forward_s=fpl, adjoint_s=bpl, grad_c2_rel_diff_vs_fp64=rel(gpl, g64)),
        speedup_vs_plain=dict(fp64=(fpl + bpl) / (f64 + b64), fp32=(fpl + bpl) / (f32 + b32)),
        forward_variant=tuned,
        lanes={k: dict(forward=plans[k].lanes, adjoint=plans[k].adjoint_lanes)
               for k in ("f64", "f32")},
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS if achieved else None,
                      traffic=prof["bytes_per_launch"] / adj_launch_s / 1e9 if prof else None,
                      traffic_bytes_per_launch=prof["bytes_per_launch"] if prof else None,
                      traffic_profile=prof["profile"] if prof else None,
                      kernel=adj_kernel, avg_launch_us=adj_launch_s * 1e6, launches=adj_n,
                      algorithmic_bytes_per_launch=adj_bytes / max(adj_n, 1),
                      lanes=1),
    )
    return rec_out


def problem_3d():
    """The 384^3 FD8 workload's inputs: c^2, the perturbed c^2 the misfit's
    data come from, H at the stability limit of the faster of the two, the
    8 Ricker point sources and the receivers."""
    import numpy as np
    from paper_1907_11771_amd.plan import scheme_weights
    from synth import fields, workloads

    cfg = workloads.CONFIG_3D
    n, R = cfg["n"], cfg["n_rhs"]
    steps, w, _ = scheme_weights(cfg["scheme"])
    cs = fields.bandlimited_lognormal_speed(n, seed=cfg["speed_seed"], kmax=cfg["kmax"])
    c2 = cs * cs
    g_obs = np.log(fields.bandlimited_lognormal_speed(n, seed=cfg["data_seed"],
                                                      kmax=cfg["kmax"], sigma=1.0))
    c2_obs = c2 * np.exp(0.1 * g_obs)
    del g_obs
    c_top = float(np.sqrt(max(c2.max(), c2_obs.max())))
    H = workloads.stable_H(workloads.ISB_ORDER8_K6, c_top, 1.0 / n, 3, workloads.SIGMA_FD8)
    src = fields.ricker_source_3d(n, workloads.sources_3d(n, R, cfg["source_seed"]))
    rec = fields.plane_receivers_3d(n, cfg["receivers"])
    return dict(cfg=cfg, n=n, R=R, steps=steps, w=w, c2=c2, c2_obs=c2_obs, c_top=c_top, H=H,
                src=src, rec=rec)


def make_plan_3d(pb, dtype, rhs, c2_host, variant=0, receivers=False):
    import torch
    from paper_1907_11771_amd import binding as B
    from paper_1907_11771_amd.plan import GBSPlan
    n, src, rec = pb["n"], pb["src"], pb["rec"]
    pl = GBSPlan(B.ACOUSTIC3D, (n, n, n), 8, pb["steps"], pb["w"], pb["H"], fd_order=8,
                 n_rhs=len(rhs), dtype=dtype, c2_field=torch.from_numpy(c2_host).to("cuda:0"),
                 c_max=pb["c_top"], device=torch.device("cuda:0"))
    if variant:
        pl.set_variant(variant)
    pts = [src["points"][r] for r in rhs]
    pl.set_sources(list(range(len(rhs))), [z * n * n + y * n + x for z, y, x in pts],
                   [src["weight"]] * len(rhs), src["f0"], src["delay"])
    if receivers:
        pl.set_receivers([i for i in range(len(rhs)) for _ in rec],
                         [z * n * n + y * n + x for _ in rhs for z, y, x in rec])
    return pl


def forward_3d_leg(nm, variant=0, pb=None):
    """The 384^3 FD8 forward, all 8 right-hand sides in one plan: FP32
    stepping with the FP64 combination and the same ``nm`` macro steps in
    FP64 (the FP32 pressure error is stated against it), and the plain FP64
    form (one streaming launch per sequence per leap-frog step) per macro
    step."""
    import torch
    from paper_1907_11771_amd import binding as B
    pb = pb or problem_3d()
    n, R = pb["n"], pb["R"]
    dev = torch.device("cuda:0")

    def release():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    res, finals = {}, {}
    for dtype in (torch.float32, torch.float64):
        pl = make_plan_3d(pb, dtype, range(R), pb["c2"], variant)
        y = torch.zeros((R, 4, n, n, n), dtype=dtype, device=dev)
        pl.step(y, y, n_macro=1)
        y.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        pl.step(y, y, n_macro=nm)
        torch.cuda.synchronize()
        res[dtype] = time.perf_counter() - t
        finals[dtype] = y[:, 0].cpu().double()
        print("acoustic3d forward %s: %.3f s for %d macro steps" % (dtype, res[dtype], nm),
              file=sys.stderr, flush=True)
        del pl, y
        release()
    # the plain FP64 form (a few macro steps suffice: the cost per macro step
    # is constant)
    n_plain = min(nm, 3)
    pl = make_plan_3d(pb, torch.float64, range(R), pb["c2"])
    pl.set_variant(B.VARIANT_PLAIN)
    y = torch.zeros((R, 4, n, n, n), dtype=torch.float64, device=dev)
    pl.step(y, y, n_macro=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    pl.step(y, y, n_macro=n_plain)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t) * 1e3 / n_plain
    del pl, y
    release()
    t32, t64 = res[torch.float32], res[torch.float64]
    err = float((finals[torch.float32] - finals[torch.float64]).abs().max()
                / finals[torch.float64].abs().max())
    upd = n ** 3 * R * (1 + sum(pb["steps"])) * nm
    return dict(
        updates_per_s=upd / t32, ms_per_step=t32 * 1e3 / nm, steps=nm, dtype="f32",
        config=dict(workload=pb["cfg"]["name"], grid=[n, n, n], n_rhs=R, fd_order=8),
        fp64_ms_per_step=t64 * 1e3 / nm,
        fp32_max_rel_err_vs_fp64_pressure=err,
        plain_fp64_ms_per_step=plain_ms,
        speedup_vs_plain=dict(fp64=plain_ms / (t64 * 1e3 / nm), fp32=plain_ms / (t32 * 1e3 / nm)))


def bench_3d(args):
    """384^3 FD8 acoustic, 8 right-hand sides (one Ricker point source each).
    Forward: forward_3d_leg.  Gradient: receiver misfit against data from a
    perturbed c^2 (FP64, all 8 right-hand sides), forward + checkpointed
    adjoint in FP32 stepping, run in groups of right-hand sides so that
    checkpoints, recomputed states and the adjoint's levels fit in HBM; the
    FP32 gradient of the first group is compared with the FP64 one."""
    import numpy as np
    import torch
    from paper_1907_11771_amd.autograd import receiver_traces

    pb = problem_3d()
    cfg, n, R = pb["cfg"], pb["n"], pb["R"]
    nm = cfg["n_macro"] if args.steps == 500 else args.steps
    ck = cfg["checkpoint_every"]
    c2, c2_obs, rec = pb["c2"], pb["c2_obs"], pb["rec"]
    dev = torch.device("cuda:0")
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log("acoustic3d: fields ready, H = %.6g" % pb["H"])

    def make(dtype, rhs, c2_host, receivers=False):
        return make_plan_3d(pb, dtype, rhs, c2_host, args.variant, receivers)

    def release():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    leg = forward_3d_leg(nm, args.variant, pb)
    line = dict(
        metric="grid-pt RHS updates/s", value=leg["updates_per_s"], unit="grid-pt RHS updates/s",
        n_gpus=1, steps=nm, warmup=1, ms_per_step=leg["ms_per_step"], higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic", config=leg["config"],
        fp64_ms_per_step=leg["fp64_ms_per_step"],
        fp32_max_rel_err_vs_fp64_pressure=leg["fp32_max_rel_err_vs_fp64_pressure"],
        plain_fp64_ms_per_step=leg["plain_fp64_ms_per_step"],
        speedup_vs_plain=leg["speedup_vs_plain"])
    if args.no_gradient:
        print(json.dumps(line), flush=True)
        return

    # data: receiver traces of the perturbed model, FP64, all right-hand sides
    parts = []
    for s0 in range(0, R, 4):
        pl = make(torch.float64, range(s0, s0 + 4), c2_obs, receivers=True)
        with torch.no_grad():
            y0 = torch.zeros((4, 4, n, n, n), dtype=torch.float64, device=dev)
            parts.append(receiver_traces(pl, y0, pl.c2_field, nm, checkpoint_every=nm))
        del pl, y0
        release()
    data = torch.cat(parts, dim=1)
    nrec = len(rec)
    log("acoustic3d: data ready")

    def gradient(dtype, rhs):
        pl = make(dtype, rhs, c2, receivers=True)
        y0 = torch.zeros((len(rhs), 4, n, n, n), dtype=dtype, device=dev, requires_grad=True)
        c2v = torch.from_numpy(c2).to(dev, dtype).requires_grad_(True)
        d = data[:, [r * nrec + i for r in rhs for i in range(nrec)]]
        d = d.contiguous()
        torch.cuda.synchronize()
        t = time.perf_counter()
        tr = receiver_traces(pl, y0, c2v, nm, checkpoint_every=ck)
        loss = 0.5 * ((tr.double() - d) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g = c2v.grad.double().clone()
        del pl, y0, c2v, tr
        release()
        log("acoustic3d gradient %s rhs %s: forward %.2f s, adjoint %.2f s"
            % (dtype, list(rhs), t1 - t, t2 - t1))
        return t1 - t, t2 - t1, g, float(loss.detach())

    # right-hand sides per plan: as many as fit in HBM.  Per right-hand side
    # of S bytes (one state): the forward workspace (an FP64 accumulator and
    # two levels of each of the six sequences, 14 S), the adjoint workspace
    # (N_max + 2 levels and two FP64 states, 18 S), the checkpoints and one
    # segment's recomputed states (n / ck + ck), and a few states besides
    free, _ = torch.cuda.mem_get_info(dev)

    def per_rhs(dtype):
        b = torch.empty((), dtype=dtype).element_size()
        return (14 + 18 + nm // ck + ck + 4) * 4 * n ** 3 * b

    group = next(g for g in (8, 4, 2, 1) if g * per_rhs(torch.float32) <= 0.85 * free)
    fw = bw = 0.0
    for s0 in range(0, R, group):
        a, b_, g, _ = gradient(torch.float32, list(range(s0, s0 + group)))
        fw, bw = fw + a, bw + b_
        del g
    # the error statement: right-hand side 0 alone in FP32 and FP64
    a32, b32, g32, _ = gradient(torch.float32, [0])
    a64, b64, g64, _ = gradient(torch.float64, [0])
    grad_err = float((g32 - g64).norm() / g64.norm()) if g64.norm() > 0 else None
    line["gradient"] = dict(receivers_per_rhs=nrec, checkpoint_every=ck, rhs_per_group=group,
                            fp32_forward_s=fw, fp32_adjoint_s=bw,
                            fp32_forward_s_rhs0=a32, fp32_adjoint_s_rhs0=b32,
                            fp64_forward_s_rhs0=a64, fp64_adjoint_s_rhs0=b64,
                            grad_c2_rel_err_fp32_vs_fp64_rhs0=grad_err)
    print(json.dumps(line), flush=True)


def bench_oneway(args):
    """The paper's experiment (Sect. 4.1) on the GPU: u_t + u_x = 0 on [0,1)
    with the Fourier derivative, u(x,0) = (1 - cos 2 pi x)/2, one revolution
    at 0.99 of each method's limit (n = ceil(pi M / (0.99 ISB)) steps of
    1/n), refined over M; the error is max |u_n - u(., 1)| against the
    analytic solution u(x, 1) = u(x, 0).  Methods: GBS_{8,6}, GBS_{12,8}
    (FP64 weights from the exact rationals) and RK4; the normalised step is
    H over the evaluations per step per core (N_max + 1 for the folded
    sequences, 4 for RK4)."""
    import math
    import torch
    from paper_1907_11771_amd import binding as B
    from paper_1907_11771_amd.plan import GBSPlan, scheme_weights
    from synth import fields, schemes

    dev = torch.device("cuda:0")
    ms = (16, 32, 64, 128, 256, 512, 1024)
    rows = []
    t_all = time.perf_counter()
    for sch in (schemes.GBS_8_6, schemes.GBS_12_8, None):
        if sch is None:
            name, isb, per_core, evals = "rk4", 2 * math.sqrt(2), 4, 4
            steps, w, p = [2, 4, 6, 8], None, 8
        else:
            steps, w, isb = scheme_weights(sch)
            name, p = sch["name"], sch["p"]
            per_core, evals = max(steps) + 1, 1 + sum(steps)
        for m in ms:
            n = math.ceil(math.pi * m / (0.99 * isb))
            u0 = torch.from_numpy(fields.oneway_initial(m)[None]).to(dev)
            if sch is None:
                plan = GBSPlan(B.ADVECT1D, (m,), 8, *scheme_weights(schemes.ORDER8_K6)[:2],
                               1e-9, fd_order=B.FD_SPECTRAL, device=dev)
                go = lambda: plan.rk4_step(u0, n_steps=n, h=1.0 / n)
            else:
                plan = GBSPlan(B.ADVECT1D, (m,), p, steps, w, 1.0 / n,
                               fd_order=B.FD_SPECTRAL, device=dev)
                go = lambda: plan.step(u0, n_macro=n)
            go()
            torch.cuda.synchronize()
            t = time.perf_counter()
            u = go()
            torch.cuda.synchronize()
            t = time.perf_counter() - t
            err = float((u - u0).abs().max())
            rows.append(dict(method=name, M=m, steps=n, H=1.0 / n,
                             normalised_step=1.0 / n / per_core, evaluations=n * evals,
                             error=err, seconds=t))
            print("oneway", name, m, n, err, t, flush=True)
    best = min(r["error"] for r in rows if r["method"] == "gbs_8_6")
    print(json.dumps(dict(
        metric="one-way wave, one revolution: lowest error of GBS_{8,6}", value=best,
        unit="max abs error", higher_is_better=False, n_gpus=1, dtype="f64", data="synthetic",
        config=dict(workload="oneway_spectral_sect4_1", M=list(ms), lam="0.99 ISB / pi",
                    seconds_total=time.perf_counter() - t_all),
        rows=rows)), flush=True)


def bench_rk4(args):
    """Time to solution at equal error, the extrapolated step against
    classical RK4 on the same stencil code (Sect. 3.8, App. A): 2048^2
    constant-c acoustic, FP64, a pulse plus 32 modes up to wavenumber 64; the
    extrapolated step at 0.8 of its stability limit for 100 macro steps (the
    library's autotuned blocked form), RK4 with the fewest steps found whose
    error is no larger.  Errors are taken against the same scheme at H/4
    (order 8: its own error is 4^8 times smaller), all on the GPU."""
    import math
    import torch
    from paper_1907_11771_amd import binding as B
    from paper_1907_11771_amd.plan import GBSPlan, scheme_weights
    from synth import fields, workloads

    cfg = workloads.CONFIG_ACOUSTIC2D
    n, H = cfg["n"], cfg["H"]
    nm = 100 if args.steps == 500 else args.steps
    steps, w, _ = scheme_weights(cfg["scheme"])
    dev = torch.device("cuda:0")
    y = torch.from_numpy(fields.acoustic2d_pulse_modes(n, n_modes=32, kmax=64, seed=0)[None])
    y = y.to(dev)
    T = nm * H
    plan = GBSPlan(B.ACOUSTIC2D, (n, n), 8, steps, w, H, dtype=torch.float64, device=dev)
    fine = GBSPlan(B.ACOUSTIC2D, (n, n), 8, steps, w, H / 4, dtype=torch.float64, device=dev)
    ref = fine.step(y, n_macro=4 * nm)
    scale = float(ref.abs().max())
    err = lambda a: float((a - ref).abs().max()) / scale
    out = torch.empty_like(y)
    tuned = plan.autotune(y, out, macro_steps=3, lanes=1)

    def timed(fn):
        fn()                                          # warm-up run of the same length
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    t_gbs, yg = timed(lambda: plan.step(y, out, n_macro=nm))
    e_gbs = err(yg)
    # RK4 from 0.8 of its own limit h rho <= 2 sqrt 2, refined (error ~ h^4)
    # until its error is within the extrapolated step's
    rho = math.sqrt(cfg["c2"]) * workloads.SIGMA_FD4 * n * math.sqrt(2)
    m = math.ceil(T / (0.8 * 2 * math.sqrt(2) / rho))
    out2 = torch.empty_like(y)
    e_rk, tries = err(plan.rk4_step(y, out2, n_steps=m, h=T / m)), 0
    while e_rk > e_gbs and tries < 8:
        m = math.ceil(m * max(1.03, 1.01 * (e_rk / e_gbs) ** 0.25))
        e_rk, tries = err(plan.rk4_step(y, out2, n_steps=m, h=T / m)), tries + 1
    t_rk, _ = timed(lambda: plan.rk4_step(y, out2, n_steps=m, h=T / m))
    print(json.dumps(dict(
        metric="time to solution at equal error vs RK4", value=t_gbs, unit="s",
        higher_is_better=False, n_gpus=1, steps=nm, dtype="f64", data="synthetic",
        config=dict(workload="gbs_vs_rk4_acoustic2d_2048", grid=[n, n], t_end=T,
                    initial="pulse + 32 modes, wavenumbers up to 64",
                    error="max |y - y_ref| / max |y_ref|, y_ref: same scheme at H/4",
                    autotuned=dict(variant=tuned[0], band=tuned[1], lanes=tuned[2])),
        gbs=dict(seconds=t_gbs, macro_steps=nm, rhs_evaluations=nm * (1 + sum(steps)),
                 rel_error=e_gbs),
        rk4=dict(seconds=t_rk, steps=m, rhs_evaluations=4 * m, rel_error=e_rk,
                 reached_equal_error=e_rk <= e_gbs),
        speedup=t_rk / t_gbs)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", type=int, default=0,
                    help="stepping-kernel variant (0: autotuned by the library)")
    ap.add_argument("--band", type=int, default=0,
                    help="rows per band of the temporally blocked passes (0 = default)")
    ap.add_argument("--form", type=int, default=None,
                    help="GBS_FORM_* flags of the blocked passes (gbs_plan_set_form)")
    ap.add_argument("--wave-order", type=int, default=None,
                    help="workgroup order of the blocked passes (gbs_plan_set_wave_order)")
    ap.add_argument("--workload", default="acoustic2d",
                    choices=["acoustic2d", "batch64", "adjoint1024", "acoustic3d", "rk4",
                             "oneway"],
                    help="acoustic2d: the 2048^2 FP64 workload (default); batch64: 64 "
                         "uneven instances in one batch; adjoint1024: forward + adjoint "
                         "gradient of the 1024^2 receiver misfit; acoustic3d: 384^3 FD8, "
                         "8 right-hand sides")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"],
                    help="stepping precision of the batch workload")
    ap.add_argument("--no-gradient", action="store_true",
                    help="acoustic3d: the forward runs only")
    ap.add_argument("--grid", type=int, default=0,
                    help="adjoint1024: another grid size (e.g. 2048 for counter profiles)")
    ap.add_argument("--no-lanes", action="store_true",
                    help="leave out the lanes-tuned timing of the default line")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="leave out the forward + adjoint leg of the default line")
    ap.add_argument("--no-batch", action="store_true",
                    help="leave out the batch workload's leg of the default line")
    ap.add_argument("--no-3d", action="store_true",
                    help="leave out the 3-D forward leg of the default line")
    ap.add_argument("--summarize-counters", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="print the TRAFFIC line of --kernel from rocprofv3 counter files")
    ap.add_argument("--kernel", help="kernel name for --summarize-counters")
    ap.add_argument("--last", type=int, default=0,
                    help="--summarize-counters: only the last LAST launches of the kernel")
    ap.add_argument("--counters-workload", help="workload name for --summarize-counters")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_counters:
        return summarize_counters(args)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method's data-parallel path is "
              "benchmarked on a single MI355X (--gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes_read=src.numel() * 8, copy_bytes_written=dst.numel() * 8,
                              launches=5)), flush=True)
        return

    from paper_1907_11771_amd import binding as B
    from paper_1907_11771_amd.plan import GBSPlan, scheme_weights
    from synth import fields, workloads

    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "adjoint1024":
        return bench_adjoint(args)
    if args.workload == "acoustic3d":
        return bench_3d(args)
    if args.workload == "rk4":
        return bench_rk4(args)
    if args.workload == "oneway":
        return bench_oneway(args)

    cfg = workloads.CONFIG_ACOUSTIC2D
    n = cfg["n"]
    steps, w, isb = scheme_weights(cfg["scheme"])
    y0 = fields.acoustic2d_pulse_modes(n)
    dev = torch.device("cuda:0")
    plan = GBSPlan(B.ACOUSTIC2D, (n, n), cfg["scheme"]["p"], steps, w, cfg["H"], fd_order=4,
                   dtype=torch.float64, c2=cfg["c2"], device=dev)
    y = torch.from_numpy(y0[None]).to(dev)
    out = torch.empty_like(y)
    tuned = None
    if args.variant or args.band:
        if args.variant:
            plan.set_variant(args.variant)
        if args.band:
            B.check(B.lib().gbs_plan_set_band(plan.handle, args.band))
    else:
        # the library's own autotuner picks the blocked variant and band
        # (untimed; it writes only into `out`).  One lane: the passes of a
        # macro step run one launch at a time, so that each launch's HIP-event
        # duration (the roofline figure) belongs to the form that is timed.
        tuned = plan.autotune(y, out, macro_steps=5, lanes=1)

    if args.wave_order is not None:
        B.check(B.lib().gbs_plan_set_wave_order(plan.handle, args.wave_order))
    if args.form is not None:
        B.check(B.lib().gbs_plan_set_form(plan.handle, args.form))
    plan.step(y, out, n_macro=args.warmup)
    torch.cuda.synchronize()
    # timed region: K macro steps in the tuned form, no events
    t = time.perf_counter()
    plan.step(y, out, n_macro=args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    # the roofline: the same K steps with every launch bracketed by HIP
    # events on the plan's stream (created beforehand)
    plan.set_timing(max(args.steps, 2))
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.step(y, out, n_macro=args.steps)
    torch.cuda.synchronize()
    dt_events = time.perf_counter() - t
    step_ms, step_n, aux_ms, aux_n = plan.get_timing()
    plan.set_timing(0)
    lanes_alt = None
    if tuned is not None and not args.no_lanes:
        # for information: the form the autotuner picks when it may also
        # spread the passes over several streams (overlapping launches, so
        # no per-launch roofline)
        alt = GBSPlan(B.ACOUSTIC2D, (n, n), cfg["scheme"]["p"], steps, w, cfg["H"], fd_order=4,
                      dtype=torch.float64, c2=cfg["c2"], device=dev)
        tl = alt.autotune(y, out, macro_steps=5, lanes=0)
        alt.step(y, out, n_macro=args.warmup)
        torch.cuda.synchronize()
        t = time.perf_counter()
        alt.step(y, out, n_macro=args.steps)
        torch.cuda.synchronize()
        lanes_alt = dict(variant=tl[0], band=tl[1], lanes=tl[2],
                         ms_per_step=(time.perf_counter() - t) * 1e3 / args.steps)
        del alt

    variant = plan.variant()
    kstep, kaux = kernel_names(variant, B)
    upd = plan.updates_per_macro_step() * args.steps
    sb, sl, ab, al = plan.algorithmic_bytes()
    step_bytes = sb * args.steps
    achieved = step_bytes / (step_ms * 1e-3) / 1e9
    launch_s = step_ms * 1e-3 / max(step_n, 1)
    prof = measured_traffic(kstep, cfg["name"])
    measured = prof["bytes_per_launch"] if prof else None
    traffic = measured / launch_s / 1e9 if measured else None
    rec = dict(
        metric="grid-pt RHS updates/s",
        value=upd / dt,
        unit="grid-pt RHS updates/s",
        n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=dt * 1e3 / args.steps,
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=cfg["name"], grid=[n, n], fields=3, fd_order=4,
                    scheme_order=8, sequences=steps, evals_per_macro_step=1 + sum(steps),
                    H=cfg["H"], macro_steps_timed=args.steps, kernel_variant=variant,
                    autotuned=dict(variant=tuned[0], band=tuned[1], lanes=tuned[2]) if tuned
                    else None),
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                      traffic_bytes_per_launch=measured,
                      traffic_profile=prof["profile"] if prof else None, kernel=kstep,
                      avg_launch_us=step_ms * 1e3 / max(step_n, 1), launches=step_n,
                      algorithmic_bytes_per_launch=step_bytes / max(step_n, 1)),
        # the streaming form must move 72 B per update; this is the rate those
        # bytes would need, i.e. the fraction of the streaming roofline reached
        streaming_equivalent=dict(bytes_per_update=STREAM_BYTES_PER_UPDATE,
                                  gbps=upd * STREAM_BYTES_PER_UPDATE / dt / 1e9,
                                  frac=upd * STREAM_BYTES_PER_UPDATE / dt / 1e9 / HBM_PEAK_GBS),
        ms_per_step_with_events=dt_events * 1e3 / args.steps,
        tuned_with_lanes=lanes_alt,
        aux_kernel=dict(kernel=kaux, avg_launch_us=aux_ms * 1e3 / max(aux_n, 1),
                        gbps=ab * args.steps / (aux_ms * 1e-3) / 1e9 if aux_ms else None),
    )
    del plan, y, out
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        # the metric's second half: forward + adjoint time at fixed error
        # against the plain form, with the adjoint pass kernel's roofline
        rec["fwd_adj"] = adjoint_leg()
    if not args.no_batch:
        # the batch workload (64 uneven instances, one graph-replayed batch)
        # in FP64 and FP32 stepping over its 100 macro steps
        inputs = batch_inputs()
        nb = workloads.CONFIG_BATCH["n_macro"]
        b64 = batch_leg(nb, 2, "f64", inputs=inputs)
        b32 = batch_leg(nb, 2, "f32", plain=False, inputs=inputs)
        b32["plain_fp64_ms_per_step"] = b64["plain_fp64_ms_per_step"]
        b32["speedup_vs_plain_fp64"] = b64["plain_fp64_ms_per_step"] / b32["ms_per_step"]
        rec["batch64"] = dict(f64=b64, f32=b32)
        del inputs
    if not args.no_3d:
        # the 384^3 FD8 forward with 8 right-hand sides (FP32 stepping, FP64
        # for the error statement, the plain FP64 form)
        rec["acoustic3d"] = forward_3d_leg(LEG_3D_MACRO_STEPS)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(cfg, y0)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
