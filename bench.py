"""Benchmark of the batched dense contraction on one MI355X.

Workload: K = 3 operators of 56 x 56, E = 2^20 elements, u ~ U(-1, 1),
D ~ N(0, 1/56), seed 0 -- both storage layouts (element-major, DOF-major)
and both FP32-tolerance precisions (fp32, bf16x3).  One step is one pass of
the hot path over that batch: for each of the four (layout, precision)
problems, resolve its transformation record and run the contraction.

The records are chosen three ways and each is timed:
  untuned  -- the default record (16-element tile, no LDS prefetch, no unroll)
  autotuned -- the exhaustive autotuner's winner (tuning runs untimed)
  learned  -- the cost model's pick, when a trained picker is available
`value` is the throughput of the learned pick if available, otherwise of the
autotuned records.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from paper_1405_7470_amd import inputs, lpx

K, NP, E = 3, 56, 1 << 20
PROBLEMS = [("em", "fp32"), ("dm", "fp32"), ("em", "bf16x3"), ("dm", "bf16x3")]
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2516.6 / 3, "bf16": 2516.6}
PEAK_HBM_GBS = 8000.0
FLOP = 2 * K * E * NP * NP                      # one contraction
BYTES = 4 * (E * NP + K * E * NP + K * NP * NP)  # read u, D once; write out once


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock budget of the oracle's bounded sample")
    return ap.parse_args()


def roof_tflops(precision):
    ai = FLOP / BYTES
    return min(PEAK_TFLOPS[precision], ai * PEAK_HBM_GBS / 1000.0)


def time_steps(work, recs, steps, warmup, stream):
    """Runs `steps` timed passes over all problems; returns (ms per step,
    per-problem mean kernel microseconds from events on the launch stream)."""
    for _ in range(warmup):
        for key, (D, u, out) in work.items():
            lpx.contract(D, u, out=out, layout=key[0], record=recs[key], stream=stream)
    torch.cuda.synchronize()
    evs = {key: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(steps)] for key in work}
    t0 = time.perf_counter()
    for s in range(steps):
        for key, (D, u, out) in work.items():
            a, b = evs[key][s]
            a.record(stream)
            lpx.contract(D, u, out=out, layout=key[0], record=recs[key], stream=stream)
            b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = {key: 1000.0 * sum(a.elapsed_time(b) for a, b in evs[key]) / steps for key in work}
    return 1000.0 * wall / steps, per


def cpu_baseline(seconds):
    """The FP64 oracle on the host cores over a bounded sample of the same
    workload (element-major, fp32): chunks of 4096 elements until the time
    budget is spent."""
    import oracle
    D, u = inputs.contraction_inputs(K, NP, E, seed=0, layout="em")
    chunk = 4096
    done = 0
    t0 = time.perf_counter()
    while done < E and time.perf_counter() - t0 < seconds:
        n = min(chunk, E - done)
        oracle.contract(D, u, "em", "fp32", done, n)
        done += n
    dt = time.perf_counter() - t0
    flop = 2 * K * done * NP * NP
    return {"value": flop / dt / 1e12, "unit": "TFLOP/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"elements [0, {done}) of E={E}, K={K}, Np={NP}, element-major, fp32 "
                      f"products with fp64 accumulation, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the contraction "
              "shards over elements with no exchange, but multi-GPU runs are not part of "
              "this build", file=sys.stderr)
        sys.exit(2)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    work = {}
    for layout, prec in PROBLEMS:
        if layout not in {k[0] for k in work}:
            D, u = inputs.contraction_inputs(K, NP, E, seed=0, layout=layout)
            Dd, ud = torch.from_numpy(D).cuda(), torch.from_numpy(u).cuda()
        else:
            Dd, ud = next((w[0], w[1]) for k, w in work.items() if k[0] == layout)
        out = torch.empty(lpx.out_shape(K, NP, E, layout), device="cuda")
        work[(layout, prec)] = (Dd, ud, out)
    torch.cuda.synchronize()

    untuned = {key: lpx.default_record(key[1]) for key in work}
    tuned, tune_times = {}, {}
    for key, (D, u, out) in work.items():
        tuned[key], tune_times[key] = lpx.autotune(D, u, out, key[0], key[1], warmup=2, reps=5,
                                                   stream=stream)
    learned = None  # filled once a trained cost model is available

    results = {}
    for name, recs in (("untuned", untuned), ("autotuned", tuned), ("learned", learned)):
        if recs is None:
            results[name] = None
            continue
        ms, per = time_steps(work, recs, args.steps, args.warmup, stream)
        results[name] = {
            "ms_per_step": ms,
            "tflops": len(work) * FLOP / (ms * 1e-3) / 1e12,
            "per_problem": {f"{k[0]}/{k[1]}": {
                "record": lpx.describe(recs[k]), "us": per[k],
                "tflops": FLOP / (per[k] * 1e-6) / 1e12,
                "gbs": BYTES / (per[k] * 1e-6) / 1e9,
                "pct_roof": 100.0 * FLOP / (per[k] * 1e-6) / 1e12 / roof_tflops(k[1])}
                for k in work}}
    primary = results["learned"] or results["autotuned"]
    # dominant kernel of the primary records: the problem with the most time
    dom_key = max(primary["per_problem"], key=lambda k: primary["per_problem"][k]["us"])
    dom = primary["per_problem"][dom_key]
    dom_prec = dom_key.split("/")[1]
    if PEAK_TFLOPS[dom_prec] <= FLOP / BYTES * PEAK_HBM_GBS / 1000.0:
        roofline = {"bound": "mfma", "achieved": dom["tflops"], "peak": PEAK_TFLOPS[dom_prec],
                    "unit": "TFLOP/s"}
    else:
        roofline = {"bound": "hbm", "achieved": dom["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roofline["frac"] = roofline["achieved"] / roofline["peak"]
    roofline["traffic"] = None
    roofline["kernel"] = f"contraction {dom_key} {dom['record']}"

    line = {
        "metric": "TFLOP/s and % roofline: learned-pick vs autotuned vs untuned, same tol",
        "value": primary["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": primary["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched dense contraction out[k,e,i]=sum_j D[k,i,j] u[e,j], "
                               "K=3, Np=56, E=2^20, layouts em+dm, precisions fp32+bf16x3",
                   "selection": "learned" if results["learned"] else "autotuned"},
        "roofline": roofline,
        "variants": results,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
