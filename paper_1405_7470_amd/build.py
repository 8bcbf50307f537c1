"""Build liblpx.so (all HIP sources for gfx950) in-tree.

Every source under csrc/ is compiled with hipcc for gfx950 (the kernel
instance units once per i-block bound) into
``_build/`` at the repository root, then linked into
``paper_1405_7470_amd/liblpx.so``.  Run as ``python -m
paper_1405_7470_amd.build``.
"""
import concurrent.futures as cf
import glob
import re
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "liblpx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = "gfx950"
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


INSTANCE_UNIT = re.compile(r"contract_\w+_(em|dm)\.hip$")
NT_BOUNDS = (8, 4, 2)  # each instance unit is compiled once per i-block bound


def _compile(job):
    src, defs = job
    tag = "".join("." + d.split("=")[1] for d in defs)
    obj = os.path.join(BUILD, os.path.basename(src) + tag + ".o")
    cmd = [HIPCC, *CFLAGS, *("-D" + d for d in defs), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature;
    # that line is expected and dropped.
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip():
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = True, jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    # the kernel-instance units take longest: start them first
    units = [(f, (f"LPX_NT={nt}",)) for nt in NT_BOUNDS for f in srcs if INSTANCE_UNIT.search(f)]
    units += [(f, ()) for f in srcs if not INSTANCE_UNIT.search(f)]
    jobs = jobs or min(len(units), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", flush=True)
    return LIB


if __name__ == "__main__":
    build()
