"""Summaries of rocprofv3 output for the contraction kernels.

Two summaries, both short text files meant to be kept next to the numbers
they support:

* ``stats``: the top kernels of a ``--kernel-trace --stats`` run (calls,
  average and total duration) from its ``*_kernel_stats.csv``.
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
            f"{ntmax}, {rec.tile_e}, {rec.prefetch}, {unroll}>(lpx::kern::ContractArgs)")


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


def write_stats(csv_path, out, cmd, title, top=25):
    with open(csv_path, newline="") as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    with open(out, "w") as fh:
        fh.write(f"# {title}\n\n")
        fh.write(f"Command: `{cmd}`\n\n")
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
        write_stats(args.csv, args.out, args.cmd, args.title)
    else:
        rows, ff, fw = traffic(args.fetch, args.write, args.copy_bytes)
        write_traffic(args.out, rows, ff, fw, args.copy_bytes, args.cmd_fetch, args.cmd_write,
                      args.title)


if __name__ == "__main__":
    main()
