"""Build the gfx950 HIP library ``libdegraf_flow.so`` in-tree with hipcc.

Every ``csrc/*.hip`` file is compiled separately (in parallel) and linked into one shared
library next to this file.  All device code is built with packed-FP32 instruction selection
disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdegraf_flow.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-I" + CSRC]
# The tracker's batched and single-pair forms are separate template instantiations whose outputs
# are bit-identical.  With implicit contraction the optimiser may fuse a * b + c in one of them and
# not in the other, so these sources are built with -ffp-contract=off and write every fused
# multiply-add out (fmaf / fma): the same operations in every instantiation by construction.
NO_CONTRACT_PREFIX = "track"


def _flags(src: str) -> list:
    extra = ["-ffp-contract=off"] if os.path.basename(src).startswith(NO_CONTRACT_PREFIX) else []
    return CFLAGS + extra


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *_flags(src), "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if out.strip():
        print(out, file=sys.stderr)
    return obj


PEAKS_SRC = os.path.join(HERE, "probes", "peaks.hip")
PEAKS_LIB = os.path.join(HERE, "probes", "libdgf_peaks.so")


def build_peaks() -> str:
    """The achievable-peak probes the benchmark uses (a library of their own)."""
    tmp = PEAKS_LIB + ".tmp"
    cmd = [HIPCC, *CFLAGS, "-shared", PEAKS_SRC, "-o", tmp]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for the peak probes:\n" + p.stdout + p.stderr)
    os.replace(tmp, PEAKS_LIB)
    return PEAKS_LIB


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        peaks = ex.submit(build_peaks)
        objs = list(ex.map(_compile, srcs))
        peaks.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
