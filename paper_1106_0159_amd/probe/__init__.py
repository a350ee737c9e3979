"""Binding of the throughput probes (libsht_probe.so, sht_probe.h): attained
instruction rates for the benchmark's roofline, beside the nominal peaks.
Benchmark instrumentation only; the transform library does not contain it."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(os.path.dirname(_HERE), "libsht_probe.so")
KINDS = {"fp64_fma": 0, "fp32_mfma_16x16x4": 1, "bf16_mfma_16x16x32": 2,
         "fp32_mfma_with_fp64_fma": 3}  # sht_probe.h
EXPORTS = ("sht_probe_flops", "sht_probe_run")

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        I = ctypes.c_int
        L.sht_probe_flops.restype = ctypes.c_double
        L.sht_probe_flops.argtypes = [I, I, I]
        L.sht_probe_run.restype = I
        L.sht_probe_run.argtypes = [I, I, I, ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def rate(kind: str, blocks: int = 8192, iters: int = 4000, device="cuda") -> dict:
    """Attained TFLOP/s of one probe (one warm-up launch, one timed with HIP
    events on torch's current stream, where the probe is launched)."""
    import torch
    k = KINDS[kind]
    flops = lib().sht_probe_flops(k, blocks, iters)
    if flops <= 0:
        raise ValueError("invalid probe arguments")
    out = torch.empty(blocks * 256, dtype=torch.float64, device=device)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if lib().sht_probe_run(k, blocks, iters, out.data_ptr(), s) != 0:
        raise RuntimeError("sht_probe_run failed")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    if lib().sht_probe_run(k, blocks, iters, out.data_ptr(), s) != 0:
        raise RuntimeError("sht_probe_run failed")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"kind": kind, "blocks": blocks, "iters": iters, "flops": flops, "ms": ms, "tflops": flops / ms / 1e9}


def coexec(blocks: int = 8192, iters: int = 4000, device="cuda") -> dict:
    """Whether FP32 matrix instructions and FP64 FMAs overlap: the interleaved
    probe's time against the FP32 matrix probe at iters plus the FP64 FMA
    probe at 8 x iters (the same work apart).  overlap = (separate sum -
    interleaved) / the shorter of the two (0: the times add, 1: full overlap)."""
    mf = rate("fp32_mfma_16x16x4", blocks, iters, device)
    fm = rate("fp64_fma", blocks, 8 * iters, device)
    both = rate("fp32_mfma_with_fp64_fma", blocks, iters, device)
    sep = mf["ms"] + fm["ms"]
    return {"blocks": blocks, "iters": iters, "mfma_ms": mf["ms"], "fma64_ms": fm["ms"], "separate_sum_ms": sep,
            "interleaved_ms": both["ms"], "overlap": (sep - both["ms"]) / min(mf["ms"], fm["ms"])}
