"""Benchmark: extrapolated GBS macro steps of the 2-D acoustic workload
(2048^2 periodic grid, FP64, FD4, order-8 scheme over N = 2,4,...,12) on one
MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One "step" is one macro step: all six GBS sequences (forward Euler, N_j
leap-frog steps, averaging) and the FP64 weighted combination, i.e.
1 + sum N_j = 43 RHS evaluations per grid point.  Prints one JSON line.
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
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by
# the plain-copy calibration) for the kernel as it is now; see profiles/.  An
# entry must be removed when its kernel changes.
MEASURED_TRAFFIC_BYTES_PER_LAUNCH = {
    "gbs::pass2d<double, 4, 7, false, 1>": 1.605e9,   # profiles/pass2d_acoustic2d_2048_fd4_f64.txt
}


def kernel_names(variant, B):
    step = {B.VARIANT_TEMPORAL: "gbs::pass2d<double, 4, 7, false, 1>",
            B.VARIANT_TEMPORAL4: "gbs::pass2d<double, 4, 4, false, 1>",
            B.VARIANT_TEMPORAL_S5: "gbs::pass2d<double, 4, 5, true, 1>",
            B.VARIANT_TEMPORAL_S6: "gbs::pass2d<double, 4, 6, true, 1>",
            B.VARIANT_TEMPORAL_WG4: "gbs::pass2d<double, 4, 7, false, 4>",
            B.VARIANT_TEMPORAL_WG8: "gbs::pass2d<double, 4, 7, false, 8>",
            B.VARIANT_FLAT: "gbs::lf_kernel<double, 4, 2>"}.get(variant,
                                                              "gbs::lf_march2d<double, 4, ...>")
    temporal = variant in (B.VARIANT_TEMPORAL, B.VARIANT_TEMPORAL4, B.VARIANT_TEMPORAL_S5,
                           B.VARIANT_TEMPORAL_S6, B.VARIANT_TEMPORAL_WG4, B.VARIANT_TEMPORAL_WG8)
    aux = "gbs::combine_kernel<double>" if temporal else "gbs::first_kernel<double, 4, 2>"
    return step, aux


def cpu_baseline(cfg, y0):
    """The oracle (NumPy FP64, one thread) on one macro step of the same grid."""
    from fractions import Fraction
    from oracle import gbs as G
    from oracle import operators as OP
    from oracle import weights as W
    sch = cfg["scheme"]
    exact = W.weights(sch["p"], sch["steps"], sch["free_idx"], [Fraction(x) for x in sch["c_free"]])
    steps, c = list(sch["steps"]), W.to_fp64(exact)
    op = OP.Acoustic((cfg["n"], cfg["n"]), c2=cfg["c2"], r=cfg["r"])
    t = time.perf_counter()
    G.macro_step(op, 0.0, y0, cfg["H"], steps, c)
    dt = time.perf_counter() - t
    updates = cfg["n"] * cfg["n"] * (1 + sum(steps))
    return dict(value=updates / dt, unit="grid-pt RHS updates/s", cores=1, kind="oracle",
                sample="1 macro step of the same 2048^2 FP64 workload (43 RHS sweeps), "
                       "%.1f s, NumPy single thread" % dt)


def bench_batch(args):
    """64 uneven instances advanced in one batch (graph-replayed macro steps,
    autotuned variant and band), against the plain FP64 form (one streaming
    launch per sequence per leap-frog step, instance by instance)."""
    import numpy as np
    import torch
    from paper_1907_11771_amd import binding as B
    from paper_1907_11771_amd.plan import GBSBatch, GBSPlan, scheme_weights
    from synth import workloads

    cfg = workloads.CONFIG_BATCH
    steps, w, _ = scheme_weights(cfg["scheme"])
    dev = torch.device("cuda:0")
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    inst = workloads.batch_instances(cfg)
    rng = np.random.default_rng(7)
    y0 = [rng.standard_normal((1, 3, n, n)) for n, _, _ in inst]
    spec = [dict(n=(n, n), H=H, c2_field=torch.from_numpy(c * c).to(dev), c_max=float(c.max()))
            for n, c, H in inst]
    batch = GBSBatch(spec, 8, steps, w, dtype=dtype, device=dev)
    tune = [torch.from_numpy(a).to(dev, dtype) for a in y0]
    variant, band = batch.autotune(tune, macro_steps=1)
    del tune
    batch.set_graph(True)
    ys = [torch.from_numpy(a).to(dev, dtype) for a in y0]
    batch.step(ys, n_macro=max(args.warmup, 1))
    ys = [torch.from_numpy(a).to(dev, dtype) for a in y0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    batch.step(ys, n_macro=args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    upd = batch.updates_per_macro_step() * args.steps

    # accuracy of this run against the FP64 batch after the same steps
    err = None
    if dtype == torch.float32:
        ref = GBSBatch(spec, 8, steps, w, dtype=torch.float64, device=dev)
        ref.set_variant(variant, band)
        yr = [torch.from_numpy(a).to(dev) for a in y0]
        ref.step(yr, n_macro=args.steps)
        err = max(float((a.double() - b).abs().max() / b.abs().max()) for a, b in zip(ys, yr))
        del ref, yr

    # the plain FP64 form on the same instances (a few macro steps, per macro step)
    plain_steps = 3
    plain_s = 0.0
    for (n, c, H), a in zip(inst, y0):
        pl = GBSPlan(B.ACOUSTIC2D, (n, n), 8, steps, w, H, dtype=torch.float64,
                     c2_field=torch.from_numpy(c * c).to(dev), c_max=float(c.max()), device=dev)
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
    rec = dict(
        metric="grid-pt RHS updates/s", value=upd / dt, unit="grid-pt RHS updates/s",
        n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=dt * 1e3 / args.steps,
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype=args.dtype,
        data="synthetic",
        config=dict(workload=cfg["name"], instances=len(inst),
                    sizes=sorted(set(n for n, _, _ in inst)), points=sum(n * n for n, _, _ in inst),
                    evals_per_macro_step=1 + sum(steps), graph=True,
                    autotuned=dict(variant=variant, band=band)),
        plain_fp64_ms_per_step=plain_ms,
        speedup_vs_plain_fp64=plain_ms / (dt * 1e3 / args.steps),
        max_rel_err_vs_fp64=err,
    )
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", type=int, default=0,
                    help="stepping-kernel variant (0 = the library's choice)")
    ap.add_argument("--band", type=int, default=0,
                    help="rows per band of the temporally blocked passes (0 = default)")
    ap.add_argument("--workload", default="acoustic2d",
                    choices=["acoustic2d", "batch64"],
                    help="acoustic2d: the 2048^2 FP64 workload (default); batch64: 64 "
                         "uneven instances in one batch")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"],
                    help="stepping precision of the batch workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
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

    cfg = workloads.CONFIG_ACOUSTIC2D
    n = cfg["n"]
    steps, w, isb = scheme_weights(cfg["scheme"])
    y0 = fields.acoustic2d_pulse_modes(n)
    dev = torch.device("cuda:0")
    plan = GBSPlan(B.ACOUSTIC2D, (n, n), cfg["scheme"]["p"], steps, w, cfg["H"], fd_order=4,
                   dtype=torch.float64, c2=cfg["c2"], device=dev)
    if args.variant:
        plan.set_variant(args.variant)
    if args.band:
        B.check(B.lib().gbs_plan_set_band(plan.handle, args.band))
    y = torch.from_numpy(y0[None]).to(dev)
    out = torch.empty_like(y)

    plan.step(y, out, n_macro=args.warmup)
    torch.cuda.synchronize()
    # timed region: K macro steps; every launch is bracketed by HIP events on
    # the plan's stream (events created beforehand)
    plan.set_timing(max(args.steps, 2))
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.step(y, out, n_macro=args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    step_ms, step_n, aux_ms, aux_n = plan.get_timing()
    plan.set_timing(0)
    # the same K steps without events, to show what the events cost
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.step(y, out, n_macro=args.steps)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t

    variant = plan.variant()
    kstep, kaux = kernel_names(variant, B)
    upd = plan.updates_per_macro_step() * args.steps
    sb, sl, ab, al = plan.algorithmic_bytes()
    step_bytes = sb * args.steps
    achieved = step_bytes / (step_ms * 1e-3) / 1e9
    launch_s = step_ms * 1e-3 / max(step_n, 1)
    measured = MEASURED_TRAFFIC_BYTES_PER_LAUNCH.get(kstep)
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
                    H=cfg["H"], macro_steps_timed=args.steps, kernel_variant=variant),
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                      traffic_bytes_per_launch=measured, kernel=kstep,
                      avg_launch_us=step_ms * 1e3 / max(step_n, 1), launches=step_n,
                      algorithmic_bytes_per_launch=step_bytes / max(step_n, 1)),
        # the streaming form must move 72 B per update; this is the rate those
        # bytes would need, i.e. the fraction of the streaming roofline reached
        streaming_equivalent=dict(bytes_per_update=STREAM_BYTES_PER_UPDATE,
                                  gbps=upd * STREAM_BYTES_PER_UPDATE / dt / 1e9,
                                  frac=upd * STREAM_BYTES_PER_UPDATE / dt / 1e9 / HBM_PEAK_GBS),
        ms_per_step_without_events=dt_plain * 1e3 / args.steps,
        aux_kernel=dict(kernel=kaux, avg_launch_us=aux_ms * 1e3 / max(aux_n, 1),
                        gbps=ab * args.steps / (aux_ms * 1e-3) / 1e9 if aux_ms else None),
    )
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(cfg, y0)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
