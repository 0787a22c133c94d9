"""Compile the HIP library libcptr.so for gfx950 (in-tree).

Setup kernels whose results feed integer decisions (decoupling, AMG setup)
are compiled with floating-point contraction off so that their evaluation
order is exactly the one written in the source; the solve-phase kernels use
the compiler's default contraction."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcptr.so")

SOURCES = {
    "k_common.hip": [],
    "k_decouple.hip": ["-ffp-contract=off"],
    "k_amg_setup.hip": ["-ffp-contract=off"],
    "k_vcycle.hip": [],
    "k_bilu.hip": [],
    "k_krylov.hip": [],
    "k_condense.hip": [],
    "k_learned.hip": ["-ffp-contract=off"],
    "k_probe.hip": [],
    "k_blocktri.hip": [],
    "host.cpp": [],
}

BASE_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for p in ("/opt/rocm/bin/hipcc",):
        if os.path.exists(p):
            return p
    return "hipcc"


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *BASE_FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = int(os.environ.get("MAX_JOBS", "8"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        futs = {ex.submit(_compile, s, f): s for s, f in SOURCES.items()}
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
