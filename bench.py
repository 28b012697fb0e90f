"""Benchmark: extrapolated GBS macro steps of the 2-D acoustic workload
(2048^2 periodic grid, FP64, FD4, order-8 scheme over N = 2,4,...,12) on one
MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One "step" is one macro step: the shared first evaluation, all leap-frog
sweeps of the six sequences, the averaging and the FP64 combination
(1 + sum N_j = 43 RHS evaluations per grid point).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s


def lf_bytes_per_macro_step(steps, points, fields, b):
    """Algorithmic bytes of the leap-frog launches of one macro step
    (streaming form): a step that stores its level reads y_{s-1}, y_s and
    writes y_{s+1} (3 F b per point); a sequence's last step reads y_{N-1},
    y_N and writes (first to finish) or reads and writes (the others) the
    FP64 accumulator, or writes y_out (the last)."""
    order = sorted(steps)
    tot = 0
    for r, n in enumerate(order):
        tot += (n - 1) * 3 * fields * b * points
        last = 2 * fields * b
        if r == 0:
            last += fields * 8
        elif r == len(order) - 1:
            last += fields * 8 + fields * b
        else:
            last += 2 * fields * 8
        tot += last * points
    return tot


def first_bytes_per_macro_step(k, points, fields, b):
    """Shared first evaluation: reads y_0, writes y_1 of every sequence."""
    return (1 + k) * fields * b * points


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
                sample="1 macro step of the same 2048^2 FP64 workload (43 sweeps), %.1f s" % dt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method's data-parallel path is "
              "benchmarked on a single MI355X (--gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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

    cfg = workloads.CONFIG_ACOUSTIC2D
    n = cfg["n"]
    steps, w, isb = scheme_weights(cfg["scheme"])
    y0 = fields.acoustic2d_pulse_modes(n)
    dev = torch.device("cuda:0")
    plan = GBSPlan(B.ACOUSTIC2D, (n, n), cfg["scheme"]["p"], steps, w, cfg["H"], fd_order=4,
                   dtype=torch.float64, c2=cfg["c2"], device=dev)
    y = torch.from_numpy(y0[None]).to(dev)
    out = torch.empty_like(y)

    plan.step(y, out, n_macro=args.warmup)
    torch.cuda.synchronize()
    # timed region: K macro steps, every launch bracketed by HIP events on the
    # plan's stream (created beforehand)
    plan.set_timing(max(args.steps, 2))
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.step(y, out, n_macro=args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    lf_ms, lf_n, first_ms, first_n = plan.get_timing()
    plan.set_timing(0)
    # the same K steps without events, to show what the events cost
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.step(y, out, n_macro=args.steps)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t

    upd = plan.updates_per_macro_step() * args.steps
    pts = n * n
    lf_bytes = lf_bytes_per_macro_step(steps, pts, 3, 8) * args.steps
    achieved = lf_bytes / (lf_ms * 1e-3) / 1e9
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
                    H=cfg["H"], macro_steps_timed=args.steps),
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=None,
                      kernel="lf_kernel<double, 4, 2>",
                      avg_launch_us=lf_ms * 1e3 / max(lf_n, 1), launches=lf_n,
                      algorithmic_bytes_per_launch=lf_bytes / max(lf_n, 1)),
        ms_per_step_without_events=dt_plain * 1e3 / args.steps,
        first_kernel=dict(avg_launch_us=first_ms * 1e3 / max(first_n, 1),
                          gbps=first_bytes_per_macro_step(len(steps), pts, 3, 8) * args.steps
                          / (first_ms * 1e-3) / 1e9 if first_ms else None),
    )
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(cfg, y0)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
