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

Besides the main line: the autotuner's sweep of every record per problem,
the small parity workload (K = 3, Np = 20, E = 4096, untuned) timed on the
GPU, dense GEMM in three precisions, the 512-instance ragged batch (one
persistent graph replay, 512 separate launches, and 512 launches captured in
one graph), and the CPU leg: the FP64 oracle timed on the host cores over
bounded samples (all cores and one thread), which also reports the
normwise error of the GPU results against the oracle on sampled outputs.

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
SMALL = (3, 20, 4096)                           # the small parity workload, element-major
SAMPLE_STARTS = (0, E // 2 + 13, E - 256)       # element chunks checked against the oracle
SAMPLE_LEN = 256


def progress(msg):
    """A progress line on stderr (long profiled runs show they are alive)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock budget of the oracle's bounded sample (all cores)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the GEMM and ragged-batch side measurements")
    ap.add_argument("--model", default=None, help="picker model file (default: the packaged one)")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the side measurements (GEMM, ragged batch, dG volume and "
                         "surface, Coulomb) and print them as one JSON line (for profiling)")
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


def sweep_table(key, times):
    """The autotuner's timing of every record of one problem (enumeration
    order): [tile_e, prefetch, unroll, order, median us, GB/s, % of roofline]."""
    recs = lpx.enumerate_records(K, NP, E, key[0], key[1])
    rows = []
    for r, t in zip(recs, times):
        if not math.isfinite(t):
            continue
        s = t * 1e-6
        rows.append([r.tile_e, r.prefetch, r.unroll, r.order, round(t, 2),
                     round(BYTES / s / 1e9, 1),
                     round(100.0 * FLOP / s / 1e12 / roof_tflops(key[1]), 2)])
    return rows


def small_case(stream):
    """The small parity workload (K = 3, Np = 20, E = 4096, element-major,
    untuned record) on the GPU: median event time of 50 launches (the
    launch includes the record's D-arrangement pre-pass).  Returns the
    timing and the host inputs and output for the CPU leg's check."""
    Kc, Npc, Ec = SMALL
    D, u = inputs.contraction_inputs(Kc, Npc, Ec, seed=0)
    Dd, ud = torch.from_numpy(D).cuda(), torch.from_numpy(u).cuda()
    out = torch.empty((Kc, Ec, Npc), device="cuda")
    t = _event_time(lambda: lpx.contract(Dd, ud, out=out, layout="em", record=None,
                                         stream=stream), 50, stream)
    flop = 2 * Kc * Ec * Npc * Npc
    res = {"workload": f"K={Kc} Np={Npc} E={Ec} em fp32, untuned record", "us": t * 1e6,
           "tflops": flop / t / 1e12}
    return res, (D, u, out.cpu().numpy())


def gemm_tiles(prec, tiles, M, N):
    """The tiling lpx_gemm runs for a record's GEMM tiles (0 = default)."""
    if tuple(tiles) != (0, 0, 0):
        return tuple(tiles)
    if prec == "fp32":
        return (128, 128, 32)
    if prec == "bf16x3" and -(-M // 256) * -(-N // 256) >= 256:
        return (256, 256, 32)
    return (128, 128, 64)


def extras(stream, learned_picker=None):
    """Side measurements of the other hot-path rows: dense GEMM (the
    degenerate case) in three precisions, and the 512-instance ragged batch
    as one graph replay vs 512 separate launches vs 512 launches captured in
    one graph.  Returns (results, host samples for the CPU leg's check)."""
    res = {"gemm": [], "batch": None}
    samples = {"gemm": []}
    for (M, N, Kd) in ((4096, 4096, 4096), (8192, 1024, 4096)):
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        A = torch.randn((M, Kd), device="cuda", generator=g)
        B = torch.randn((Kd, N), device="cuda", generator=g)
        C = torch.empty((M, N), device="cuda")
        rows = [0, M // 2 + 17, M - 1]
        entry = {"shape": (M, N, Kd), "A": A[rows].cpu().numpy(), "B": B.cpu().numpy(),
                 "rows": rows, "C": {}}
        # the whole call: for BF16 / BF16X3 it includes the split of the FP32
        # operands into bf16 planes (two HBM-bound pre-passes)
        for prec, tiles in (("fp32", (128, 128, 64)), ("bf16", (0, 0, 0)),
                            ("bf16", (256, 256, 64)), ("bf16x3", (0, 0, 0))):
            rec = lpx.record(prec, gemm=tiles)
            t = _event_time(lambda: lpx.gemm(A, B, C, record=rec, stream=stream), 5, stream)
            tf = 2 * M * N * Kd / t / 1e12
            res["gemm"].append({"shape": [M, N, Kd], "precision": prec,
                                "tiles": list(gemm_tiles(prec, tiles, M, N)),
                                "us": t * 1e6, "tflops": tf,
                                "pct_peak": 100 * tf / PEAK_TFLOPS[prec]})
            entry["C"].setdefault(prec, C[rows].cpu().numpy())
        samples["gemm"].append(entry)
        # context, not this library: torch.matmul (the vendor GEMM library)
        # on operands already in bf16, same shape
        Ab, Bb = A.to(torch.bfloat16), B.to(torch.bfloat16)
        t = _event_time(lambda: torch.matmul(Ab, Bb), 5, stream)
        res.setdefault("gemm_context", []).append(
            {"shape": [M, N, Kd], "what": "torch.matmul, bf16 operands (vendor library)",
             "us": t * 1e6, "tflops": 2 * M * N * Kd / t / 1e12})
        del A, B, C, Ab, Bb
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
    else:  # the default record is valid for every shape
        recs = [lpx.default_record("fp32")] * len(shapes)
        how = "default fp32 record"
    flop = sum(2 * K * Ei * Np * Np for Np, Ei in shapes)
    nbytes = sum(4 * (Ei * Np + K * Ei * Np + K * Np * Np) for Np, Ei in shapes)
    roof = sum(max(2 * K * Ei * Np * Np / (PEAK_TFLOPS["fp32"] * 1e12),
                   4 * (Ei * Np + K * Ei * Np + K * Np * Np) / (PEAK_HBM_GBS * 1e9))
               for Np, Ei in shapes)
    bt = lpx.Batch(items, recs, stream=stream)
    t_graph = _event_time(lambda: bt.submit(stream=stream), 5, stream)
    torch.cuda.synchronize()
    batch_out = [o.clone() for (_, _, o, _) in items[:8]]
    binfo = bt.info()
    bt.destroy()
    t_sep = _event_time(lambda: [lpx.contract(D, u, out=o, record=r, stream=stream)
                                 for (D, u, o, l), r in zip(items, recs)], 3, stream)
    # 512 launches captured in one graph (lpx_contract_noalloc allocates
    # nothing, so it can be captured): the fair comparison for the persistent
    # kernel, since both pay one graph launch
    t_cap, same = None, None
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for (D, u, o, l), r in zip(items, recs):  # warm the per-kernel caches
                lpx.contract_noalloc(D, u, o, layout=l, record=r, stream=side)
        side.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            for (D, u, o, l), r in zip(items, recs):
                lpx.contract_noalloc(D, u, o, layout=l, record=r, stream=side)
        torch.cuda.synchronize()
        t_cap = _event_time(graph.replay, 5, stream)
        torch.cuda.synchronize()
        same = all(torch.equal(o, b) for (_, _, o, _), b in zip(items[:8], batch_out))
        del graph
    except Exception as exc:  # a side measurement never hides the rest
        same = repr(exc)
    # records tuned for the batch itself (lpx_batch_tune: each (K, Np)
    # group timed as a batch with every candidate record)
    t0 = time.perf_counter()
    trecs = lpx.batch_tune(items, "fp32", warmup=1, reps=3, stream=stream)
    tune_s = time.perf_counter() - t0
    bt = lpx.Batch(items, trecs, stream=stream)
    t_tuned = _event_time(lambda: bt.submit(stream=stream), 5, stream)
    torch.cuda.synchronize()
    tinfo = bt.info()
    tuned_same = all(torch.equal(o, b) for (_, _, o, _), b in zip(items[:8], batch_out))
    bt.destroy()
    chosen = {}
    for (D, _, _, _), r in zip(items, trecs):
        chosen[str(D.shape[1])] = lpx.describe(r)
    res["batch_tuned"] = {"graph_us": t_tuned * 1e6, "graph_tflops": flop / t_tuned / 1e12,
                          "graph_pct_roof": 100 * roof / t_tuned, "tune_s": tune_s,
                          "graph_kernels": tinfo["kernels"], "records_by_Np": chosen,
                          "equals_learned_batch": tuned_same}
    res["batch"] = {"instances": len(shapes), "records": how, "gflop": flop / 1e9,
                    "gbytes": nbytes / 1e9,
                    "graph_us": t_graph * 1e6, "separate_us": t_sep * 1e6,
                    "captured_launches_us": t_cap * 1e6 if t_cap else None,
                    "graph_tflops": flop / t_graph / 1e12,
                    "separate_tflops": flop / t_sep / 1e12,
                    "captured_launches_tflops": flop / t_cap / 1e12 if t_cap else None,
                    "captured_equals_batch": same,
                    "roofline_us": roof * 1e6, "graph_pct_roof": 100 * roof / t_graph,
                    "graph_kernels": binfo["kernels"], "graph_workgroups": binfo["grid"]}
    return res, samples


COULOMB_NT, COULOMB_NS = 1 << 20, 1 << 15
# v_sub x3, v_mul, v_fmac x3, v_cmp, v_cndmask at the full FP32 rate and
# v_rsq_f32 at a quarter of it: 13 VALU lane-slots per pair.  FP32 vector
# peak 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 FMA lanes per clock, so
# 256 x 128 x 2.4e9 lane-slots per second
COULOMB_SLOTS_PER_PAIR = 13
COULOMB_PEAK_PAIRS = 256 * 128 * 2.4e9 / COULOMB_SLOTS_PER_PAIR


def coulomb_extras(stream):
    """The 3D Coulomb potential at 2^20 targets x 2^15 sources, every
    variant in both storage layouts (median of 3 launches each)."""
    res = {"nt": COULOMB_NT, "ns": COULOMB_NS, "unit": "Mpairs/s",
           "alu_peak_mpairs": COULOMB_PEAK_PAIRS / 1e6, "layouts": {}}
    pairs = COULOMB_NT * COULOMB_NS
    for layout in ("em", "dm"):
        tg, sr = inputs.coulomb_inputs(COULOMB_NT, COULOMB_NS, seed=0, layout=layout)
        tgd, srd = torch.from_numpy(tg).cuda(), torch.from_numpy(sr).cuda()
        phi = torch.empty(COULOMB_NT, device="cuda")
        sweep = []
        for rec in lpx.coulomb_records():
            t = _event_time(lambda: lpx.coulomb(tgd, srd, phi, layout=layout, record=rec,
                                                stream=stream), 3, stream)
            sweep.append([rec.tile_e * 16, rec.prefetch, rec.unroll, round(t * 1e6, 1),
                          round(pairs / t / 1e6, 0)])
        best = max(sweep, key=lambda r: r[4])
        res["layouts"]["aos" if layout == "em" else "soa"] = {
            "best": {"source_tile": best[0], "prefetch": best[1], "targets_per_thread": best[2],
                     "us": best[3], "mpairs_per_s": best[4],
                     "frac_alu_peak": best[4] * 1e6 / COULOMB_PEAK_PAIRS},
            "sweep_columns": ["source_tile", "prefetch", "targets_per_thread", "us", "Mpairs/s"],
            "sweep": sweep}
        del tgd, srd, phi
    return res


def dg_extras(stream):
    """The dG volume term at K = 3, Np = 56, E = 2^20 (the contraction plus
    per-element 3 x 3 geometric factors applied by the store waves)."""
    Kd, Npd, Ed = K, NP, E
    flop = 2 * Kd * Ed * Npd * Npd + 2 * Kd * Kd * Ed * Npd
    nbytes = 4 * (Ed * Npd + Kd * Ed * Npd + Kd * Npd * Npd + Kd * Kd * Ed)
    out = {"workload": f"K={Kd} Np={Npd} E={Ed}", "gflop": flop / 1e9, "gbytes": nbytes / 1e9,
           "runs": []}
    for layout in ("em", "dm"):
        D, u, G = inputs.dg_volume_inputs(Kd, Npd, Ed, seed=0, layout=layout)
        Dd, ud, Gd = (torch.from_numpy(x).cuda() for x in (D, u, G))
        o = torch.empty(lpx.out_shape(Kd, Npd, Ed, layout), device="cuda")
        for prec, tile, pf in (("fp32", 64, 14), ("fp32", 64, 10), ("bf16x3", 64, 14),
                               ("bf16x3", 32, 14)):
            rec = lpx.record(prec, tile, pf, 1)
            t = _event_time(lambda: lpx.dg_volume(Dd, ud, Gd, out=o, layout=layout, record=rec,
                                                  stream=stream), 5, stream)
            tf = flop / t / 1e12
            roof = min(PEAK_TFLOPS[prec], flop / nbytes * PEAK_HBM_GBS / 1000.0)
            out["runs"].append({"layout": layout, "record": lpx.describe(rec), "us": t * 1e6,
                                "tflops": tf, "gbs": nbytes / t / 1e9,
                                "pct_roof": 100 * tf / roof})
        del Dd, ud, Gd, o
    return out


def surface_extras(stream):
    """The dG surface (lift) term at Np = 56, 4 faces of 21 nodes, E = 2^20:
    every variant in FP32 and bf16x3, both layouts (median of 5)."""
    Nps, nf, nfp, Es = 56, 4, 21, E
    M = nf * nfp
    flop = 2 * Nps * M * Es
    nbytes = 4 * (Es * M + Es * nf + Es * Nps + Nps * M)
    out = {"workload": f"Np={Nps} nf={nf} nfp={nfp} E={Es}", "gflop": flop / 1e9,
           "gbytes": nbytes / 1e9, "runs": []}
    for layout in ("em", "dm"):
        L, f, s = inputs.dg_surface_inputs(Nps, nf, nfp, Es, seed=0, layout=layout)
        Ld, fd, sd = (torch.from_numpy(x).cuda() for x in (L, f, s))
        o = torch.empty((Es, Nps) if layout == "em" else (Nps, Es), device="cuda")
        for prec in ("fp32", "bf16x3"):
            roof = min(PEAK_TFLOPS[prec], flop / nbytes * PEAK_HBM_GBS / 1000.0)
            for rec in lpx.surface_records(prec):
                t = _event_time(lambda: lpx.dg_surface(Ld, fd, sd, nf, out=o, layout=layout,
                                                       record=rec, stream=stream), 5, stream)
                tf = flop / t / 1e12
                out["runs"].append({"layout": layout, "record": lpx.describe(rec), "us": t * 1e6,
                                    "tflops": tf, "gbs": nbytes / t / 1e9,
                                    "pct_roof": 100 * tf / roof})
        del Ld, fd, sd, o
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(seconds, data, gpu_chunks, small, extra_samples):
    """The FP64 oracle on the host cores.  Timed: a bounded sample of the
    step (rounds of 2048 more elements of each of the four problems until
    the budget is spent) on all cores, a shorter one on one thread, and the
    small workload (median of 3) on all cores and on one thread.  Untimed:
    the oracle's results for sampled outputs of the GPU run, compared with
    them (normwise relative error, the parity metric of the tests)."""
    import oracle
    nthreads = oracle.threads()

    def sample_rate(budget):
        chunk, done = 2048, 0
        t0 = time.perf_counter()
        while done < E and time.perf_counter() - t0 < budget:
            n = min(chunk, E - done)
            for layout, prec in PROBLEMS:
                D, u = data[layout]
                oracle.contract(D, u, layout, prec, done, n)
            done += n
        dt = time.perf_counter() - t0
        return len(PROBLEMS) * 2 * K * done * NP * NP / dt / 1e12, done, dt

    value, done, dt = sample_rate(seconds)
    oracle.set_threads(1)
    try:
        v1, done1, dt1 = sample_rate(seconds / 4)
        D, u, _ = small
        ts1 = sorted(_timed(lambda: oracle.contract(D, u, "em", "fp32")) for _ in range(3))[1]
    finally:
        oracle.set_threads(nthreads)
    D, u, _ = small
    tsn = sorted(_timed(lambda: oracle.contract(D, u, "em", "fp32")) for _ in range(3))[1]
    base = {"value": value, "unit": "TFLOP/s", "cores": nthreads, "kind": "oracle",
            "sample": f"elements [0, {done}) of E={E} for each of em/fp32, dm/fp32, "
                      f"em/bf16x3, dm/bf16x3 (K={K}, Np={NP}), fp64 accumulation, "
                      f"{dt:.1f} s on {nthreads} threads",
            "single_thread": {"value": v1, "unit": "TFLOP/s",
                              "sample": f"elements [0, {done1}), {dt1:.1f} s"},
            "small_workload_ms": {"threads_1": ts1 * 1e3, f"threads_{nthreads}": tsn * 1e3},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}

    parity = {}
    for key, chunks in gpu_chunks.items():
        layout, prec = key.split("/")
        D, u = data[layout]
        errs = []
        for s0, got in chunks:
            ref = oracle.contract(D, u, layout, "fp32", s0, got.shape[1])
            errs.append(oracle.rel_err(got, ref))
        parity[key] = max(errs)
    D, u, out = small
    parity["small_workload/fp32"] = oracle.rel_err(out, oracle.contract(D, u, "em", "fp32"))
    for entry in (extra_samples or {}).get("gemm", []):
        M, N, Kd = entry["shape"]
        # timing sample: 192 rows of A (the three sampled rows repeated; the
        # oracle's time does not depend on the values), 16 on one thread
        At = np.tile(entry["A"], (64, 1))
        gflop = 2.0 * N * Kd
        t_all = _timed(lambda: oracle.gemm(At, entry["B"], "fp32"))
        oracle.set_threads(1)
        try:
            t_one = _timed(lambda: oracle.gemm(At[:16], entry["B"], "fp32"))
        finally:
            oracle.set_threads(nthreads)
        base.setdefault("gemm", []).append({
            "shape": [M, N, Kd], "unit": "TFLOP/s",
            "value": gflop * At.shape[0] / t_all / 1e12,
            "single_thread": gflop * 16 / t_one / 1e12,
            "sample": f"{At.shape[0]} rows of C, fp64 accumulation, {t_all:.2f} s on "
                      f"{nthreads} threads; 16 rows, {t_one:.2f} s on one thread"})
        for prec, C in entry["C"].items():
            ref = oracle.gemm(entry["A"], entry["B"], "fp32")
            parity[f"gemm {M}x{N}x{Kd}/{prec}"] = oracle.rel_err(C, ref)
    return base, {"metric": "max|gpu - oracle| / max|oracle| on sampled outputs",
                  "sampled": f"elements {list(SAMPLE_STARTS)} + {SAMPLE_LEN} of each problem; "
                             "the whole small workload; GEMM rows 0, M/2+17, M-1",
                  "rel_err": parity,
                  "tolerance": {"fp32": 1e-5, "bf16x3": 1e-5, "bf16": 2e-2}}


def _timed(fn):
    t0 = time.perf_counter()
    fn()
    return time.perf_counter() - t0


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the contraction "
              "shards over elements with no exchange, but multi-GPU runs are not part of "
              "this build", file=sys.stderr)
        sys.exit(2)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    if args.extras_only:
        from paper_1405_7470_amd import picker as picker_mod
        model = args.model or picker_mod.MODEL_PATH
        pk = lpx.Picker(model) if os.path.exists(model) else None
        line = {"extras": extras(stream, learned_picker=pk)[0]}
        progress("GEMM and batch done")
        for name, fn in (("coulomb", coulomb_extras), ("dg_volume", dg_extras),
                         ("dg_surface", surface_extras)):
            line["extras"][name] = fn(stream)
            progress(f"{name} done")
        print(json.dumps(line), flush=True)
        return
    work, host = {}, {}
    for layout, prec in PROBLEMS:
        if layout not in host:
            host[layout] = inputs.contraction_inputs(K, NP, E, seed=0, layout=layout)
            D, u = host[layout]
            Dd, ud = torch.from_numpy(D).cuda(), torch.from_numpy(u).cuda()
        else:
            Dd, ud = next((w[0], w[1]) for k, w in work.items() if k[0] == layout)
        out = torch.empty(lpx.out_shape(K, NP, E, layout), device="cuda")
        work[(layout, prec)] = (Dd, ud, out)
    torch.cuda.synchronize()

    untuned = {key: lpx.default_record(key[1]) for key in work}
    tuned, sweeps = {}, {}
    # A 512 MiB buffer is overwritten before every timed launch: u (235 MB)
    # would otherwise stay in the 256 MB last-level cache between repeats of
    # one problem, which the timed steps (four problems in turn) never see.
    # With the flush the tuner's picks run 0.852 ms per step, without it
    # 0.894 ms (same machine, same run).
    flush = torch.empty((512 << 20) // 4, device="cuda")
    for key, (D, u, out) in work.items():
        tuned[key], times = lpx.autotune(D, u, out, key[0], key[1], warmup=2, reps=5,
                                         stream=stream, flush=flush)
        sweeps[f"{key[0]}/{key[1]}"] = sweep_table(key, times)
        progress(f"tuned {key[0]}/{key[1]}")
    del flush
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
        progress(f"timed {name} records")
        results[name] = {
            "ms_per_step": ms,
            "tflops": len(work) * FLOP / (ms * 1e-3) / 1e12,
            "per_problem": {f"{k[0]}/{k[1]}": {
                "record": lpx.describe(recs[k]), "us": per[k],
                "tflops": FLOP / (per[k] * 1e-6) / 1e12,
                "gbs": BYTES / (per[k] * 1e-6) / 1e9,
                "pct_roof": 100.0 * FLOP / (per[k] * 1e-6) / 1e12 / roof_tflops(k[1])}
                for k in work}}
    # the outputs now hold the primary records' results (timed last)
    gpu_chunks = {}
    for (layout, prec), (_, _, out) in work.items():
        chunks = []
        for s0 in SAMPLE_STARTS:
            c = out[:, s0:s0 + SAMPLE_LEN, :] if layout == "em" else \
                out[:, :, s0:s0 + SAMPLE_LEN].transpose(1, 2)
            chunks.append((s0, c.double().cpu().numpy()))
        gpu_chunks[f"{layout}/{prec}"] = chunks
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
        "dtype": "fp32+bf16x3",
        "data": "synthetic",
        "config": {"workload": "batched dense contraction out[k,e,i]=sum_j D[k,i,j] u[e,j], "
                               "K=3, Np=56, E=2^20, layouts em+dm, precisions fp32+bf16x3",
                   "selection": "learned" if results["learned"] else "autotuned"},
        "roofline": roofline,
        "variants": results,
        "sweep": {"columns": ["tile_e", "prefetch", "unroll", "order", "us", "GBps",
                              "pct_roof"],
                  "note": "autotuner medians (5 reps, a 512 MiB cache flush before each) "
                          "of every supported record",
                  "problems": sweeps},
    }
    if pick_info:
        line["picker"] = pick_info
    line["hbm_copy"] = hbm_copy(stream)
    small_res, small_host = small_case(stream)
    line["small_workload"] = small_res
    ex_samples = None
    if not args.no_extras:
        try:
            line["extras"], ex_samples = extras(
                stream, learned_picker=(pk if learned is not None else None))
            progress("GEMM and batch done")
        except Exception as exc:  # side measurements never hide the main line
            line["extras"] = {"error": repr(exc)}
    if not args.no_extras:
        for name, fn in (("coulomb", coulomb_extras), ("dg_volume", dg_extras),
                         ("dg_surface", surface_extras)):
            try:
                line["extras"][name] = fn(stream)
                progress(f"{name} done")
            except Exception as exc:  # side measurements never hide the main line
                line["extras"][name] = {"error": repr(exc)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["parity"] = cpu_leg(args.cpu_seconds, host, gpu_chunks,
                                                       small_host, ex_samples)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
