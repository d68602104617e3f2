"""Builds libpdbo.so for gfx950 in-tree with hipcc.

    python -m paper_2509_21064_amd.build [-v]

Every HIP source under csrc/ is compiled to objects under _build/ (in
parallel; dense.hip in four parts) and linked into
paper_2509_21064_amd/libpdbo.so.  Always recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpdbo.so")
ARCH = os.environ.get("PDBO_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-I" + INCLUDE, "-I" + CSRC,
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

# (source, object, extra flags): dense.hip is compiled four times, each part
# instantiating one share of its kernels (part 0: everything but the step
# kernels; parts 1-3: the step kernels of one kind of g), so that the parts
# compile in parallel.
UNITS = [
    ("dense.hip", "dense_p0.o", ["-DPDBO_DENSE_PART=0"]),
    ("dense.hip", "dense_p1.o", ["-DPDBO_DENSE_PART=1"]),
    ("dense.hip", "dense_p2.o", ["-DPDBO_DENSE_PART=2"]),
    ("dense.hip", "dense_p3.o", ["-DPDBO_DENSE_PART=3"]),
    ("sparse.hip", "sparse.o", []),
    ("maxsat.hip", "maxsat.o", []),
    ("spmm.hip", "spmm.o", []),
    ("cert.hip", "cert.o", []),
    ("kcut.hip", "kcut.o", []),
    ("realw.hip", "realw.o", []),
    ("api.hip", "api.o", []),
]
SOURCES = sorted({u[0] for u in UNITS})


def _compile(unit, verbose: bool) -> str:
    src, oname, extra = unit
    obj = os.path.join(BUILD, oname)
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        msg = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    workers = max(1, min(len(UNITS), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
