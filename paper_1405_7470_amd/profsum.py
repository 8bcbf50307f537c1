"""Summaries of rocprofv3 output for the contraction kernels.

Two summaries, both short text files meant to be kept next to the numbers
they support:

* ``stats``: the top kernels of a ``--kernel-trace --stats`` run (calls,
  average and total duration) from its ``*_kernel_stats.csv``.
* ``counters``: per-dispatch averages of SQ/GRBM counters from one
  ``--pmc`` run for the contraction kernels a bench.py line names, with the
  MFMA utilisation they imply (SQ_VALU_MFMA_BUSY_CYCLES over four SIMDs
  times SQ_BUSY_CU_CYCLES).
* ``kernels``: per-dispatch counter averages of the side-workload kernels
  (GEMM, ragged batch, dG, lift, Coulomb) whose names match a pattern.
* ``traffic``: HBM bytes per launch of every contraction kernel from two
  ``--pmc`` runs (``FETCH_SIZE``, then ``WRITE_SIZE``; KiB per dispatch).
  Each counter is scaled by what it reads for the plain copy kernel
  (``stream_kernel``) of the same run, whose bytes are known, so the figures
  are HBM bytes, not counter units.

The traffic file records a hash of the contraction kernel sources; a reader
treats its figures as stale once the sources differ (``read_traffic``).

    python -m paper_1405_7470_amd.profsum stats --csv RUN_kernel_stats.csv \
        --out profiles/X.md --cmd "<the rocprofv3 command>"
    python -m paper_1405_7470_amd.profsum traffic --fetch F.csv --write W.csv \
        --copy-bytes N --out profiles/Y.txt --cmd-fetch "..." --cmd-write "..."
"""
import argparse
import csv
import hashlib
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_KERNEL = "stream_kernel"
PRECISION_CODE = {"fp32": 0, "bf16": 1, "bf16x3": 2}
LAYOUT_CODE = {"em": 0, "dm": 1}


def kernel_source_hash():
    """sha256 (first 16 hex digits) of every source that shapes a
    contraction kernel's memory traffic."""
    h = hashlib.sha256()
    names = sorted(f for f in os.listdir(CSRC)
                   if re.match(r"contract_.*\.(h|hip)$", f) or f in ("lpx_internal.h", "abi.hip"))
    for f in names:
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def contraction_kernel_name(precision, layout, Np, rec):
    """Demangled name of the kernel instance a record runs for (layout, Np)."""
    nt = (Np + 15) // 16
    ntmax = 2 if nt <= 2 else (4 if nt <= 4 else 8)
    unroll = 1 if rec.prefetch & 4 else rec.unroll  # register-D kernels are built once
    return (f"void lpx::kern::contract_kernel<{PRECISION_CODE[precision]}, {LAYOUT_CODE[layout]}, "
            f"{ntmax}, {rec.tile_e}, {rec.prefetch}, {unroll}, 0>(lpx::kern::ContractArgs)")


def _per_kernel(path, counter):
    vals = defaultdict(list)
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in vals.items()}


def traffic(fetch_csv, write_csv, copy_bytes):
    """{kernel name: (fetch KiB, write KiB, HBM bytes)} per dispatch, plus the
    two calibration factors (bytes per counter KiB)."""
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")
    copy = [k for k in f if COPY_KERNEL in k]
    if not copy or copy[0] not in w:
        raise ValueError(f"no {COPY_KERNEL} dispatch in both counter files")
    ff = copy_bytes / f[copy[0]]
    fw = copy_bytes / w[copy[0]]
    rows = {}
    for k in f:
        if k in w:
            rows[k] = (f[k], w[k], f[k] * ff + w[k] * fw)
    return rows, ff, fw


def write_traffic(out, rows, ff, fw, copy_bytes, cmd_fetch, cmd_write, title):
    with open(out, "w") as fh:
        fh.write(f"# {title}\n")
        fh.write("# HBM bytes per dispatch from two rocprofv3 --pmc runs:\n")
        fh.write(f"#   {cmd_fetch}\n#   {cmd_write}\n")
        fh.write(f"# calibration: the copy kernel moves {copy_bytes} bytes each way per dispatch;\n")
        fh.write(f"#   FETCH_SIZE scale {ff:.1f} bytes per counted KiB, "
                 f"WRITE_SIZE scale {fw:.1f} bytes per counted KiB\n")
        fh.write(f"# kernel_source_sha256 {kernel_source_hash()}\n")
        fh.write("# fetch_kib\twrite_kib\ttraffic_bytes\tkernel\n")
        for k in sorted(rows, key=lambda k: -rows[k][2]):
            fe, wr, t = rows[k]
            fh.write(f"{fe:.1f}\t{wr:.1f}\t{t:.0f}\t{k}\n")


def read_traffic(path):
    """(source hash recorded, {kernel name: HBM bytes per dispatch})."""
    src, table = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("# kernel_source_sha256"):
                src = line.split()[2]
            elif line.strip() and not line.startswith("#"):
                fe, wr, t, name = line.rstrip("\n").split("\t")
                table[name] = float(t)
    return src, table


def lookup_traffic(path, kernel):
    """HBM bytes per dispatch of `kernel` from a traffic summary, or None when
    the file is missing, the kernel is absent or the sources have changed
    since the counters were taken."""
    if not os.path.exists(path):
        return None
    src, table = read_traffic(path)
    if src != kernel_source_hash():
        return None
    return table.get(kernel)


_REC = re.compile(r"(\w+) tile_e=(\d+) prefetch=(\d+) unroll=(\d+)")


class _Rec:
    def __init__(self, desc):
        m = _REC.match(desc)
        self.precision, self.tile_e, self.prefetch, self.unroll = (
            m.group(1), int(m.group(2)), int(m.group(3)), int(m.group(4)))


def timed_region(trace_csv, kernels, steps):
    """Average duration (us) of each kernel over the last `steps` complete
    cycles in which the given kernels were dispatched back to back in this
    order (the timed steps of bench.py launch its problems round-robin)."""
    with open(trace_csv, newline="") as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [r["Kernel_Name"] for r in rows]
    n = len(kernels)
    cycles = [i for i in range(len(names) - n + 1) if names[i:i + n] == kernels]
    # the longest chain of cycles that follow one another directly
    best, cur = [], []
    for i in cycles:
        cur = cur + [i] if cur and i == cur[-1] + n else [i]
        if len(cur) >= len(best):
            best = cur
    use = best[-steps:]
    avg = []
    for k in range(n):
        d = [int(rows[i + k]["End_Timestamp"]) - int(rows[i + k]["Start_Timestamp"]) for i in use]
        avg.append(sum(d) / len(d) / 1e3 if d else float("nan"))
    return avg, len(use)


def counters(csv_path):
    """{kernel name: {counter: average per dispatch}} from a --pmc run."""
    vals = defaultdict(lambda: defaultdict(list))
    with open(csv_path, newline="") as fh:
        for r in csv.DictReader(fh):
            vals[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items()}


def write_counters(csv_path, bench_json, out, cmd, title):
    import json
    b = json.load(open(bench_json))
    sel = b["config"]["selection"]
    per = b["variants"][sel]["per_problem"]
    Np = int(re.search(r"Np=(\d+)", b["config"]["workload"]).group(1))
    table = counters(csv_path)
    names = sorted({c for k in table for c in table[k]})
    with open(out, "w") as fh:
        fh.write(f"# {title}\n\nCommand: `{cmd}`\n\n")
        fh.write("Per-dispatch averages (counters summed over the device) for the kernels of "
                 f"the {sel} records; MFMA utilisation = SQ_VALU_MFMA_BUSY_CYCLES / "
                 "(4 SIMDs x SQ_BUSY_CU_CYCLES).\n\n")
        fh.write("| problem | kernel | MFMA utilisation | " + " | ".join(names) + " |\n")
        fh.write("|---|---|---|" + "---|" * len(names) + "\n")
        for key, v in per.items():
            rec = _Rec(v["record"])
            kname = contraction_kernel_name(rec.precision, key.split("/")[0], Np, rec)
            row = table.get(kname)
            if row is None:
                continue
            util = (row.get("SQ_VALU_MFMA_BUSY_CYCLES", float("nan")) /
                    (4.0 * row.get("SQ_BUSY_CU_CYCLES", float("nan"))))
            fh.write(f"| {key} | `{kname}` | {util:.3f} | " +
                     " | ".join(f"{row.get(c, float('nan')):.4g}" for c in names) + " |\n")


def write_kernel_counters(csv_paths, out, cmds, title, pattern, top=40):
    """Per-dispatch counter averages of every kernel whose name matches
    `pattern` (the side workloads: GEMM, ragged batch, dG, lift, Coulomb),
    with the MFMA utilisation when both SQ counters are present.  Several
    --pmc runs of the same command merge into one table (one column per
    counter)."""
    table = defaultdict(dict)
    for path in csv_paths:
        for k, row in counters(path).items():
            table[k].update(row)
    rx = re.compile(pattern)
    names = sorted({c for k in table for c in table[k]})
    keys = [k for k in table if rx.search(k)][:top]
    with open(out, "w") as fh:
        fh.write(f"# {title}\n\n")
        for c in cmds:
            fh.write(f"Command: `{c}`\n\n")
        fh.write("Per-dispatch averages (counters summed over the device; a kernel's average "
                 "mixes every shape it ran on in the command).  MFMA utilisation = "
                 "SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x SQ_BUSY_CU_CYCLES).\n\n")
        util_col = "SQ_VALU_MFMA_BUSY_CYCLES" in names and "SQ_BUSY_CU_CYCLES" in names
        fh.write("| kernel |" + (" MFMA utilisation |" if util_col else "") +
                 "".join(f" {n} |" for n in names) + "\n")
        fh.write("|---|" + ("---|" if util_col else "") + "---|" * len(names) + "\n")
        for k in sorted(keys):
            row = table[k]
            cells = []
            if util_col:
                cells.append(f"{row['SQ_VALU_MFMA_BUSY_CYCLES'] / (4.0 * row['SQ_BUSY_CU_CYCLES']):.3f}"
                             if row.get("SQ_BUSY_CU_CYCLES") else "n/a")
            cells += [f"{row.get(c, float('nan')):.4g}" for c in names]
            fh.write(f"| `{k}` | " + " | ".join(cells) + " |\n")


def write_stats(csv_path, out, cmd, title, top=25, trace_csv=None, bench_json=None):
    with open(csv_path, newline="") as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    with open(out, "w") as fh:
        fh.write(f"# {title}\n\n")
        fh.write(f"Command: `{cmd}`\n\n")
        if trace_csv and bench_json:
            import json
            b = json.load(open(bench_json))
            sel = b["config"]["selection"]
            per = b["variants"][sel]["per_problem"]
            keys = list(per)
            Np = int(re.search(r"Np=(\d+)", b["config"]["workload"]).group(1))
            kern = [contraction_kernel_name(_Rec(per[k]["record"]).precision, k.split("/")[0], Np,
                                            _Rec(per[k]["record"])) for k in keys]
            avg, ncyc = timed_region(trace_csv, kern, b["steps"])
            fh.write(f"Timed steps of the {sel} records ({ncyc} cycles of the round-robin "
                     "launch sequence found in the per-dispatch trace), against the same run's "
                     "own HIP-event timing:\n\n")
            fh.write("| problem | record | kernel | trace average us | bench event us |\n"
                     "|---|---|---|---|---|\n")
            for k, name, a in zip(keys, kern, avg):
                fh.write(f"| {k} | {per[k]['record'].split(' gemm')[0]} | `{name}` | {a:.1f} | "
                         f"{per[k]['us']:.1f} |\n")
            fh.write(f"\nbench line of this run: value {b['value']:.2f} {b['unit']}, "
                     f"{b['ms_per_step']:.4f} ms per step; dominant kernel "
                     f"{b['roofline']['kernel']}\n\n")
        fh.write("All kernels of the run (an instance's average mixes every shape it was "
                 "launched on, including the ragged batch's separate launches):\n\n")
        fh.write("| kernel | calls | average us | total us | % |\n|---|---|---|---|---|\n")
        for r in rows[:top]:
            fh.write(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("--csv", required=True)
    a.add_argument("--out", required=True)
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", default="rocprofv3 kernel statistics")
    a.add_argument("--trace", default=None, help="the run's *_kernel_trace.csv")
    a.add_argument("--bench-json", default=None, help="the bench.py line of the same run")
    c = sub.add_parser("counters")
    c.add_argument("--csv", required=True)
    c.add_argument("--bench-json", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", default="SQ counters of the contraction kernels")
    k = sub.add_parser("kernels")
    k.add_argument("--csv", required=True, action="append", help="repeatable")
    k.add_argument("--out", required=True)
    k.add_argument("--cmd", required=True, action="append", help="one per --csv")
    k.add_argument("--pattern", default=".")
    k.add_argument("--title", default="Counters of the side-workload kernels")
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--cmd-fetch", required=True)
    b.add_argument("--cmd-write", required=True)
    b.add_argument("--title", default="HBM traffic per dispatch")
    args = ap.parse_args()
    if args.what == "stats":
        write_stats(args.csv, args.out, args.cmd, args.title, trace_csv=args.trace,
                    bench_json=args.bench_json)
    elif args.what == "counters":
        write_counters(args.csv, args.bench_json, args.out, args.cmd, args.title)
    elif args.what == "kernels":
        write_kernel_counters(args.csv, args.out, args.cmd, args.title, args.pattern)
    else:
        rows, ff, fw = traffic(args.fetch, args.write, args.copy_bytes)
        write_traffic(args.out, rows, ff, fw, args.copy_bytes, args.cmd_fetch, args.cmd_write,
                      args.title)


if __name__ == "__main__":
    main()
