"""Compile the HIP libraries for gfx950 in-tree with hipcc.

libsht.so        the transform library (include/sht.h)
libsht_probe.so  benchmark-only throughput probes (probe/sht_probe.h)

Each source is compiled to an object of its own, in parallel, then linked.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsht.so")
SOURCES = ["sht_abi.cpp", "sht_plan.cpp", "sht_batch.cpp", "sht_noalloc.hip", "k_legendre.hip", "k_legendre_mx.hip",
           "k_ring_fft.hip"]
PROBE_DIR = os.path.join(PKG, "probe")
PROBE_LIB = os.path.join(PKG, "libsht_probe.so")
PROBE_SOURCES = ["k_probe.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
FLAGS = COMMON + ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _compile(src: str, flags, verbose: bool) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *flags, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def _link(objs, out: str, verbose: bool) -> str:
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Always recompiles; writes paper_1106_0159_amd/libsht.so and libsht_probe.so."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = [(os.path.join(CSRC, s), FLAGS) for s in SOURCES]
    jobs += [(os.path.join(PROBE_DIR, s), COMMON + ["-I" + PROBE_DIR]) for s in PROBE_SOURCES]
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda j: _compile(j[0], j[1], verbose), jobs))
    _link(objs[: len(SOURCES)], LIB, verbose)
    _link(objs[len(SOURCES):], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
