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

from paper_1405_7470_amd import inputs, lpx, profsum

K, NP, E = 3, 56, 1 << 20
PROBLEMS = [("em", "fp32"), ("dm", "fp32"), ("em", "bf16x3"), ("dm", "bf16x3")]
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2516.6 / 3, "bf16": 2516.6}
PEAK_HBM_GBS = 8000.0
COPY_FLOATS = 1 << 26                            # 256 MiB copy: HBM reference and counter calibration
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "contract_traffic_K3_Np56_E1M.txt")
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
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the GEMM and ragged-batch side measurements")
    ap.add_argument("--model", default=None, help="picker model file (default: the packaged one)")
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


def _event_time(fn, reps, stream):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) * 1e-3)
    return sorted(ts)[len(ts) // 2]


def hbm_copy(stream):
    """Achievable HBM bandwidth on this GPU: a plain 256 MiB device copy
    (lpx_stream_probe), median of 5.  Its dispatches also calibrate the
    rocprofv3 byte counters."""
    x = torch.zeros(COPY_FLOATS, device="cuda")
    y = torch.empty(COPY_FLOATS, device="cuda")
    t = _event_time(lambda: lpx.stream_probe(x, y, 1, stream=stream), 5, stream)
    del x, y
    return {"bytes_each_way": 4 * COPY_FLOATS, "us": t * 1e6, "GBps": 8 * COPY_FLOATS / t / 1e9}


def extras(stream, learned_picker=None):
    """Side measurements of the other hot-path rows: dense GEMM (the
    degenerate case) in three precisions, and the 512-instance ragged batch
    as one graph replay vs 512 separate launches."""
    res = {"gemm": [], "batch": None}
    for (M, N, Kd) in ((4096, 4096, 4096), (8192, 1024, 4096)):
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        A = torch.randn((M, Kd), device="cuda", generator=g)
        B = torch.randn((Kd, N), device="cuda", generator=g)
        C = torch.empty((M, N), device="cuda")
        for prec, tiles in (("fp32", (128, 128, 64)), ("bf16", (128, 128, 64)),
                            ("bf16x3", (128, 128, 64))):
            rec = lpx.record(prec, gemm=tiles)
            t = _event_time(lambda: lpx.gemm(A, B, C, record=rec, stream=stream), 5, stream)
            tf = 2 * M * N * Kd / t / 1e12
            res["gemm"].append({"shape": [M, N, Kd], "precision": prec, "tiles": list(tiles),
                                "us": t * 1e6, "tflops": tf,
                                "pct_peak": 100 * tf / PEAK_TFLOPS[prec]})
        del A, B, C
    shapes = inputs.ragged_shapes(n=512, seed=0)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    items = []
    for Np, Ei in shapes:
        D = torch.randn((K, Np, Np), device="cuda", generator=g) / math.sqrt(Np)
        u = torch.rand((Ei, Np), device="cuda", generator=g) * 2 - 1
        items.append((D, u, torch.empty((K, Ei, Np), device="cuda"), "em"))
    if learned_picker is not None:
        recs = [lpx.pick_variant(K, Np, Ei, "em", "fp32", mode=lpx.PICK_LEARNED,
                                 picker=learned_picker, stream=stream) for Np, Ei in shapes]
        how = "learned"
    else:
        recs = [lpx.record("fp32", 64, 1, 2)] * len(shapes)
        how = "fixed fp32 tile_e=64 prefetch=1 unroll=2"
    flop = sum(2 * K * Ei * Np * Np for Np, Ei in shapes)
    roof = sum(max(2 * K * Ei * Np * Np / (PEAK_TFLOPS["fp32"] * 1e12),
                   4 * (Ei * Np + K * Ei * Np + K * Np * Np) / (PEAK_HBM_GBS * 1e9))
               for Np, Ei in shapes)
    bt = lpx.Batch(items, recs, stream=stream)
    t_graph = _event_time(lambda: bt.submit(stream=stream), 5, stream)
    bt.destroy()
    t_sep = _event_time(lambda: [lpx.contract(D, u, out=o, record=r, stream=stream)
                                 for (D, u, o, l), r in zip(items, recs)], 3, stream)
    res["batch"] = {"instances": len(shapes), "records": how, "gflop": flop / 1e9,
                    "graph_us": t_graph * 1e6, "separate_us": t_sep * 1e6,
                    "graph_tflops": flop / t_graph / 1e12,
                    "separate_tflops": flop / t_sep / 1e12,
                    "roofline_us": roof * 1e6, "graph_pct_roof": 100 * roof / t_graph}
    return res


def cpu_baseline(seconds):
    """The FP64 oracle on the host cores over a bounded sample of the same
    step: rounds of 2048 more elements of each of the four (layout,
    precision) problems until the time budget is spent."""
    import oracle
    data = {}
    for layout in ("em", "dm"):
        data[layout] = inputs.contraction_inputs(K, NP, E, seed=0, layout=layout)
    chunk = 2048
    done = 0
    t0 = time.perf_counter()
    while done < E and time.perf_counter() - t0 < seconds:
        n = min(chunk, E - done)
        for layout, prec in PROBLEMS:
            D, u = data[layout]
            oracle.contract(D, u, layout, prec, done, n)
        done += n
    dt = time.perf_counter() - t0
    flop = len(PROBLEMS) * 2 * K * done * NP * NP
    return {"value": flop / dt / 1e12, "unit": "TFLOP/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"elements [0, {done}) of E={E} for each of em/fp32, dm/fp32, "
                      f"em/bf16x3, dm/bf16x3 (K={K}, Np={NP}), fp64 accumulation, {dt:.1f} s"}


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
    learned, pick_info = None, None
    from paper_1405_7470_amd import picker as picker_mod
    model = args.model or picker_mod.MODEL_PATH
    if os.path.exists(model):
        pk = lpx.Picker(model)
        learned = {}
        t0 = time.perf_counter()
        for key in work:
            learned[key] = lpx.pick_variant(K, NP, E, key[0], key[1], mode=lpx.PICK_LEARNED,
                                            picker=pk, stream=stream)
        pick_info = {"model": os.path.basename(model),
                     "first_pick_us_per_problem": 1e6 * (time.perf_counter() - t0) / len(work)}

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
    dom_layout = dom_key.split("/")[0]
    dom_rec = (learned or tuned)[(dom_layout, dom_prec)]
    kname = profsum.contraction_kernel_name(dom_prec, dom_layout, NP, dom_rec)
    t = profsum.lookup_traffic(TRAFFIC_FILE, kname)
    roofline["traffic"] = t
    roofline["traffic_note"] = (
        "HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE scaled by the copy kernel"
        if t is not None else "no counter reading for this kernel at the current sources")
    roofline["algorithmic_bytes"] = BYTES
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
    if pick_info:
        line["picker"] = pick_info
    line["hbm_copy"] = hbm_copy(stream)
    if not args.no_extras:
        try:
            line["extras"] = extras(stream, learned_picker=(pk if learned is not None else None))
        except Exception as exc:  # side measurements never hide the main line
            line["extras"] = {"error": repr(exc)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
