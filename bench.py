"""Benchmark: FP64 alm2map + map2alm on HEALPix N_side=1024, lmax=mmax=2048.

One step = one map through both transforms, with inputs resident in HBM:
    alm --(Legendre synthesis)--> Delta --(ring FFT synthesis)--> map
    map --(ring FFT analysis)--> Delta^S --(Legendre analysis)--> alm'
called through the four stage entry points of the C ABI (their composition is
exactly sht_alm2map followed by sht_map2alm), with HIP events on the launch
stream between stages.  Further legs: "batched_mixed" and "batched_fp64" run
the same two transforms on a batch of 64 maps (mixed-precision and FP64
Legendre contraction); "config3" the batched Gauss-Legendre configuration
(1025 x 2049, lmax 1024, 64 maps); "small_latency" the launch-bound lmax 256
case; "serving" the continuous-batching server.
Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch N] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_MFMA_TFLOPS = 157.3  # dense FP32 matrix-core peak
PEAK_HBM_GBS = 8000.0
FLOPS_PER_TRIPLE = 8           # recurrence 4 + complex-by-real contraction 4 per (slot, l, m)
DOMINANT_SOURCES = ["paper_1106_0159_amd/csrc/k_legendre.hip", "paper_1106_0159_amd/csrc/k_device.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in DOMINANT_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_counters(stage: str) -> dict:
    """Per-launch figures from committed rocprofv3 counter runs of a Legendre stage
    (HBM bytes from FETCH_SIZE/WRITE_SIZE scaled by a plain-copy calibration, and
    executed FP64 flops from the SQ FP64 instruction counters), or {} when the
    kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return {}
    ent = rec.get(stage)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return {}
    return ent


def count_triples(geom_handle_slots: int, lmax: int, mmax: int) -> int:
    nalm = (mmax + 1) * (2 * lmax + 2 - mmax) // 2
    return geom_handle_slots * nalm


def latency(times_ms) -> dict:
    """Percentiles of the event-timed solve latency (one step or one batch)."""
    import numpy as np
    t = np.asarray(times_ms, dtype=float)
    return {"p50": float(np.percentile(t, 50)), "p99": float(np.percentile(t, 99)),
            "min": float(t.min()), "max": float(t.max()), "n": int(t.size)}


def mirror_slots(theta) -> int:
    """Number of ring slots (mirror pairs plus unpaired rings), as the library
    forms them: rings pair when |theta + theta' - pi| <= 2^-50 (two ulp of pi),
    the sum taken exactly."""
    import numpy as np
    th = sorted(float(t) for t in theta)
    pi_l = np.longdouble("3.14159265358979323846264338327950288")
    i, j, n = 0, len(th) - 1, 0
    while i <= j:
        if i == j:
            n += 1
            break
        d = float((np.longdouble(th[i]) + np.longdouble(th[j])) - pi_l)
        if abs(d) <= 2.0 ** -50:
            i += 1
            j -= 1
        elif d < 0:
            i += 1
        else:
            j -= 1
        n += 1
    return n


def cpu_baseline(g, lmax, a, mp, target_s: float = 12.0):
    """Time the oracle on a strided sample of rings (alm2map) and of m (map2alm)."""
    import numpy as np

    import oracle
    cores = oracle.get_threads()
    # calibrate with a small sample, then size the sample to about target_s in total
    rings = np.arange(0, g.nrings, 256, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.alm2map(lmax, lmax, g, a, rings=rings)
    t_r = (time.perf_counter() - t0) / len(rings)
    ms = np.arange(0, lmax + 1, 256, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.map2alm(lmax, lmax, g, mp, ms=ms)
    t_m = (time.perf_counter() - t0) / len(ms)
    k_r = max(1, min(g.nrings, int(0.5 * target_s / max(t_r, 1e-9))))
    k_m = max(1, min(lmax + 1, int(0.5 * target_s / max(t_m, 1e-9))))
    rings = np.unique(np.linspace(0, g.nrings - 1, k_r).round().astype(np.int32))
    ms = np.unique(np.linspace(0, lmax, k_m).round().astype(np.int32))
    t0 = time.perf_counter()
    oracle.alm2map(lmax, lmax, g, a, rings=rings)
    t_syn = (time.perf_counter() - t0) * g.nrings / len(rings)
    t0 = time.perf_counter()
    oracle.map2alm(lmax, lmax, g, mp, ms=ms)
    t_ana = (time.perf_counter() - t0) * (lmax + 1) / len(ms)
    # the same oracle on one thread, on a sample a quarter that size
    oracle.set_threads(1)
    try:
        r1 = rings[:: max(1, 4 * cores)] if len(rings) > 4 * cores else rings[:1]
        m1 = ms[:: max(1, 4 * cores)] if len(ms) > 4 * cores else ms[:1]
        t0 = time.perf_counter()
        oracle.alm2map(lmax, lmax, g, a, rings=r1)
        t1_syn = (time.perf_counter() - t0) * g.nrings / len(r1)
        t0 = time.perf_counter()
        oracle.map2alm(lmax, lmax, g, mp, ms=m1)
        t1_ana = (time.perf_counter() - t0) * (lmax + 1) / len(m1)
    finally:
        oracle.set_threads(cores)
    return {
        "value": 1.0 / (t_syn + t_ana),
        "unit": "maps/s",
        "cores": int(cores),
        "value_1core": 1.0 / (t1_syn + t1_ana),
        "kind": "oracle",
        "sample": (f"oracle alm2map on {len(rings)} of {g.nrings} rings (evenly spaced) and map2alm on "
                   f"{len(ms)} of {lmax + 1} m values (evenly spaced), scaled to the full map; "
                   f"est. {t_syn:.1f} s + {t_ana:.1f} s per map; value_1core: one thread on every "
                   f"{max(1, 4 * cores)}-th of those rings and m values ({len(r1)} and {len(m1)})"),
    }


def run_batch(sht, gh, g, lmax, alm, steps, warmup, flags):
    """A batch of maps through both transforms (alm -> map -> alm'), through
    the four stage entry points, HIP events on the launch stream around each
    stage.  With SHT_MIXED, Delta is kept as sht_alm2map / sht_map2alm keep
    it (the stage calls give the same bits as the combined ones): map-minor,
    [nrings][mmax+1][nmaps], in synthesis from 8 maps on, ring-major in
    analysis.  SHT_MIXED_SPLIT_BF16, a synthesis variant, goes to the
    synthesis call only.  Returns (stage ms, per-batch ms list, wall ms per
    batch, map, a_lm')."""
    import numpy as np
    import torch
    dev = alm.device
    nmaps = alm.shape[0]
    mixed = bool(flags & sht.SHT_MIXED)
    mm = mixed and nmaps >= 8
    MM = sht.SHT_DELTA_MAP_MINOR
    if mm:
        delta = torch.empty((g.nrings, lmax + 1, nmaps), dtype=torch.complex128, device=dev)
    else:
        delta = torch.empty((nmaps, g.nrings, lmax + 1), dtype=torch.complex128, device=dev)
    delta_s = torch.empty((nmaps, g.nrings, lmax + 1), dtype=torch.complex128, device=dev)
    mp = torch.zeros((nmaps, g.npix), dtype=torch.float64, device=dev)
    a_out = torch.empty_like(alm)
    ws = sht.workspace(lmax, lmax, gh, nmaps, dev, flags)
    fs = flags | (MM if mm else 0)

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        sht.alm2delta(alm, gh, lmax, lmax, out=delta, ws=ws, flags=fs)
        mark(1)
        sht.delta2map(delta, gh, lmax, out=mp, flags=MM if mm else 0)
        mark(2)
        sht.map2delta(mp, gh, lmax, out=delta_s)
        mark(3)
        sht.delta2alm(delta_s, gh, lmax, lmax, out=a_out, ws=ws, flags=flags & ~sht.SHT_MIXED_SPLIT_BF16)
        mark(4)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1000.0 / steps
    names = ["leg_syn", "fft_syn", "fft_ana", "leg_ana"]
    st = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs])) for i, n in enumerate(names)}
    batch_ms = [e[0].elapsed_time(e[4]) for e in evs]
    del delta, delta_s, ws
    return st, batch_ms, wall_ms, mp, a_out


def batch_record(nmaps, st, batch_ms, wall_ms, steps, dtype, flops_per_launch, peak, bound, kernels):
    """Throughput, stage times and the roofline of the slower Legendre stage."""
    ms = max(wall_ms, sum(st.values()))
    dom = max(("leg_syn", "leg_ana"), key=lambda n: st[n])
    achieved = flops_per_launch / (st[dom] * 1e-3) / 1e12
    return {
        "nmaps": nmaps,
        "value": nmaps * 1000.0 / ms,
        "unit": "maps/s",
        "ms_per_batch": ms,
        "latency_ms": latency(batch_ms),
        "steps": steps,
        "stages_ms": st,
        "alm2map_maps_per_s": nmaps * 1000.0 / (st["leg_syn"] + st["fft_syn"]),
        "map2alm_maps_per_s": nmaps * 1000.0 / (st["fft_ana"] + st["leg_ana"]),
        "dtype": dtype,
        "roofline": {
            "kernel": kernels[dom],
            "bound": bound,
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "flops_per_launch": flops_per_launch,
        },
    }


def fft_roofline(g, mmax, nmaps, stages_ms) -> dict:
    """Ring stages against the HBM roofline: algorithmic bytes per launch
    set = Delta (16 B per ring and m <= mmax, read in synthesis, written in
    analysis) plus the map (8 B per pixel, written / read), times the maps,
    over the event-timed stage."""
    nbytes = nmaps * (16 * g.nrings * (mmax + 1) + 8 * g.npix)
    out = {"bytes_per_launch": nbytes, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    for key, st in (("syn", "fft_syn"), ("ana", "fft_ana")):
        gbs = nbytes / (stages_ms[st] * 1e-3) / 1e9
        out[key] = {"achieved": gbs, "frac": gbs / PEAK_HBM_GBS, "ms": stages_ms[st]}
    return out


def power_law_batch(si, lmax, nmaps, config):
    import torch
    alm = torch.empty((nmaps, si.nalm(lmax, lmax)), dtype=torch.complex128, device="cuda")
    for i in range(nmaps):
        alm[i] = torch.from_numpy(si.powerlaw_alm(lmax, lmax, si.config_seed(config, i))).cuda()
    return alm


MX_KERNELS = {"leg_syn": "k_prescale_mx + k_leg_syn_mx", "leg_ana": "k_leg_ana_mx"}
F64_KERNELS = {"leg_syn": "k_prescale + k_leg_syn", "leg_ana": "k_leg_ana (+ k_ana_combine above 2048 slots)"}


def rel_per_map(x, y):
    """Relative RMS of x - y per map (rows), as a list."""
    return ((x - y).norm(dim=1) / y.norm(dim=1)).cpu().tolist()


def batched_legs(sht, si, gh, g, lmax, nmaps, steps, warmup, nslots, mp_fp64, a_fp64):
    """Batches of nmaps power-law maps on the benchmark grid, both transforms:
    "batched_mixed" (FP64 recurrence; synthesis products from three-way bf16
    splits of the FP32 operands on the bf16 matrix cores, SHT_MIXED |
    SHT_MIXED_SPLIT_BF16, the fastest mixed synthesis; analysis on the FP32
    matrix cores, SHT_MIXED; Delta and FFTs FP64) and "batched_fp64" (the
    same work in FP64).  Map 0 of the batch is the map of the plain FP64
    step: the relative RMS differences of its map and of its analysed a_lm
    to the plain results are reported, and every map of the mixed batch
    against the FP64 batch.  "variants" gives maps/s and the largest errors
    against the FP64 batch of the split products, of the FP32 products
    (SHT_MIXED alone, one FP32 l-chain) and of SHT_MIXED_FP64_SUMS (FP32
    products, synthesis block sums added in FP64)."""
    alm = power_law_batch(si, lmax, nmaps, 2)
    flops_mx = 4 * nmaps * count_triples(nslots, lmax, lmax)
    fsp = sht.SHT_MIXED | sht.SHT_MIXED_SPLIT_BF16
    st, bm, wall, mp_x, a_x = run_batch(sht, gh, g, lmax, alm, steps, warmup, fsp)
    mx = batch_record(nmaps, st, bm, wall, steps, "f64 recurrence; synthesis 3 x bf16 split products, "
                      "analysis f32 products; f32 accumulation", flops_mx, PEAK_FP32_MFMA_TFLOPS, "mfma", MX_KERNELS)
    flops_64 = FLOPS_PER_TRIPLE * nmaps * count_triples(nslots, lmax, lmax)
    st, bm, wall, mp_d, a_d = run_batch(sht, gh, g, lmax, alm, steps, warmup, 0)
    f64 = batch_record(nmaps, st, bm, wall, steps, "f64", flops_64, PEAK_FP64_VALU_TFLOPS, "alu", F64_KERNELS)
    rel = lambda x, y: (x - y).norm().item() / y.norm().item()
    f64["relrms_map0_vs_plain"] = rel(mp_d[0], mp_fp64)
    f64["relrms_alm0_vs_plain"] = rel(a_d[0], a_fp64)
    mx["relrms_map0_vs_fp64"] = rel(mp_x[0], mp_fp64)
    mx["relrms_alm0_vs_fp64"] = rel(a_x[0], a_fp64)
    e_map, e_alm = rel_per_map(mp_x, mp_d), rel_per_map(a_x, a_d)
    mx["relrms_vs_fp64_batch"] = {"map_max": max(e_map), "map_mean": sum(e_map) / nmaps,
                                  "alm_max": max(e_alm), "alm_mean": sum(e_alm) / nmaps}
    mx["speedup_vs_batched_fp64"] = mx["value"] / f64["value"]
    del mp_x, a_x

    def variant(flags, dtype):
        st, bm, wall, mp_v, a_v = run_batch(sht, gh, g, lmax, alm, steps, warmup, flags)
        rec = batch_record(nmaps, st, bm, wall, steps, dtype, flops_mx, PEAK_FP32_MFMA_TFLOPS, "mfma", MX_KERNELS)
        e_m, e_a = rel_per_map(mp_v, mp_d), rel_per_map(a_v, a_d)
        return {"value": rec["value"], "ms_per_batch": rec["ms_per_batch"], "stages_ms": rec["stages_ms"],
                "map_relrms_max": max(e_m), "map_relrms_mean": sum(e_m) / nmaps, "alm_relrms_max": max(e_a)}

    mx["variants"] = {
        "split_bf16x3": {"value": mx["value"], "map_relrms_max": mx["relrms_vs_fp64_batch"]["map_max"],
                         "alm_relrms_max": mx["relrms_vs_fp64_batch"]["alm_max"]},
        "fp32_chain": variant(sht.SHT_MIXED, "f64 recurrence, f32 products and accumulation"),
        "fp64_block_sums": variant(sht.SHT_MIXED | sht.SHT_MIXED_FP64_SUMS,
                                   "f64 recurrence, f32 products, f64 block sums"),
    }
    mx["fft_roofline"] = fft_roofline(g, lmax, nmaps, mx["stages_ms"])
    f64["fft_roofline"] = fft_roofline(g, lmax, nmaps, f64["stages_ms"])
    mx["direction"] = f64["direction"] = "alm2map+map2alm"
    return mx, f64


def config3(sht, si, steps, warmup, with_oracle):
    """The batched Gauss-Legendre configuration: 64 power-law maps on 1025
    rings x 2049 points (2049 = 3 x 683: Bluestein ring transforms), lmax =
    mmax = 1024, both transforms, mixed precision (synthesis from split bf16
    products, analysis from FP32 products) and FP64.  Errors: every
    mixed map against the FP64 map, map 0 against the oracle over every
    pixel, and the round trip against the seed a_lm (exact on this grid, so
    a property of the transforms, independent of either implementation)."""
    import numpy as np
    lmax, nmaps = 1024, 64
    g = si.gauss_legendre(lmax + 1, 2 * lmax + 1)
    gh = sht.GeomHandle(g)
    nslots = mirror_slots(g.theta)
    alm = power_law_batch(si, lmax, nmaps, 3)
    tri = count_triples(nslots, lmax, lmax)
    st, bm, wall, mp_x, a_x = run_batch(sht, gh, g, lmax, alm, steps, warmup,
                                        sht.SHT_MIXED | sht.SHT_MIXED_SPLIT_BF16)
    mx = batch_record(nmaps, st, bm, wall, steps, "f64 recurrence; synthesis 3 x bf16 split products, "
                      "analysis f32 products; f32 accumulation", 4 * nmaps * tri, PEAK_FP32_MFMA_TFLOPS, "mfma",
                      MX_KERNELS)
    st, bm, wall, mp_d, a_d = run_batch(sht, gh, g, lmax, alm, steps, warmup, 0)
    f64 = batch_record(nmaps, st, bm, wall, steps, "f64", FLOPS_PER_TRIPLE * nmaps * tri,
                       PEAK_FP64_VALU_TFLOPS, "alu", F64_KERNELS)
    e_map = rel_per_map(mp_x, mp_d)
    e_rt_x, e_rt_d = rel_per_map(a_x, alm), rel_per_map(a_d, alm)
    out = {
        "workload": "batched alm2map+map2alm, Gauss-Legendre 1025 x 2049, lmax=mmax=1024, 64 maps, power-law a_lm",
        "mixed": mx, "fp64": f64, "speedup_mixed_vs_fp64": mx["value"] / f64["value"],
        "fft_roofline": fft_roofline(g, lmax, nmaps, mx["stages_ms"]),
        "errors": {"mixed_map_vs_fp64_max": max(e_map), "mixed_map_vs_fp64_mean": float(np.mean(e_map)),
                   "mixed_roundtrip_vs_seed_max": max(e_rt_x), "fp64_roundtrip_vs_seed_max": max(e_rt_d)},
    }
    if with_oracle:
        import oracle
        a0 = alm[0].cpu().numpy()
        t0 = time.perf_counter()
        ref = oracle.alm2map(lmax, lmax, g, a0)
        m0x, m0d = mp_x[0].cpu().numpy(), mp_d[0].cpu().numpy()
        nrm = np.linalg.norm(ref)
        out["errors"]["mixed_map0_vs_oracle"] = float(np.linalg.norm(m0x - ref) / nrm)
        out["errors"]["fp64_map0_vs_oracle"] = float(np.linalg.norm(m0d - ref) / nrm)
        out["errors"]["oracle_s"] = time.perf_counter() - t0
    return out


def serving(sht, si, nreq: int, slots: int, budget_gb: float, loads=(0.5, 0.8)) -> dict:
    """Serving leg: nreq requests of the HEALPix serving mix (lmax log-uniform
    in [64, 4096], nside = lmax/2, alm2map or map2alm with equal odds, one map
    each) through the continuous-batching server.  Plans of every grid are
    built before the timed runs; inputs are resident on the device (map2alm
    takes the FP64 alm2map of its power-law a_lm).  Per precision mode: first
    every request at t = 0 (the saturation rate), then Poisson arrivals at
    fractions of that rate.  Latency is arrival to completion event."""
    import numpy as np
    import torch
    from paper_1106_0159_amd import serve

    lm, kinds, t_unit = si.serving_trace(nreq, si.config_seed(5))
    grids = {L: sht.GeomHandle(si.healpix(L // 2)) for L in sorted(set(lm.tolist()))}
    serve.Server.reserve_plans(len(grids) + 8)
    t0 = time.perf_counter()
    for L, gh in grids.items():
        sht.prepare(gh, L)
    prep_s = time.perf_counter() - t0
    print(f"[serve] {len(grids)} grids prepared in {prep_s:.1f} s, plan cache {sht.plan_cache_bytes() / 1e9:.2f} GB",
          file=sys.stderr, flush=True)
    inputs = []
    for i, (L, k) in enumerate(zip(lm.tolist(), kinds.tolist())):
        a = torch.from_numpy(si.powerlaw_alm(L, L, si.config_seed(5, i))).cuda()
        inputs.append(a if k == "alm2map" else sht.alm2map(a, grids[L], L))
    torch.cuda.synchronize()
    print(f"[serve] {nreq} request inputs resident", file=sys.stderr, flush=True)
    budget = int(budget_gb * (1 << 30))
    out = {"requests": nreq, "distinct_grids": len(grids), "slots": slots, "hbm_budget_bytes": budget,
           "lmax_range": [int(lm.min()), int(lm.max())], "alm2map_share": float(np.mean(kinds == "alm2map")),
           "prepare_s": prep_s, "plan_cache_bytes": sht.plan_cache_bytes()}

    def run(flags, rate):
        reqs = [serve.Request(k, L, grids[L], inputs[i], arrival=0.0 if rate is None else float(t_unit[i]) / rate)
                for i, (L, k) in enumerate(zip(lm.tolist(), kinds.tolist()))]
        srv = serve.Server(budget, slots, flags, keep_results=False)
        srv.run_trace(reqs)
        torch.cuda.synchronize()
        st = srv.stats()
        st["offered_per_s"] = None if rate is None else rate
        return st

    for mode, flags in (("fp64", 0), ("mixed", sht.SHT_MIXED)):
        run(flags, None)  # warm-up pass
        sat = run(flags, None)
        rows = [sat]
        rate_sat = sat["done"] / sat["span_s"]
        for f in loads:
            rows.append(run(flags, f * rate_sat))
        out[mode] = rows
        print(f"[serve] {mode}: saturation {sat['maps_per_s']:.0f} maps/s, "
              + ", ".join(f"load {r['offered_per_s']:.0f}/s p50 {r['p50_ms']:.2f} p99 {r['p99_ms']:.2f} ms"
                          for r in rows[1:]), file=sys.stderr, flush=True)
    return out


def small_latency(sht, si, calls: int = 200) -> dict:
    """The launch-bound case: alm2map alone, FP64, lmax = mmax = 256 on a
    Gauss-Legendre grid of 257 rings x 513 points, one map.  Per-call time of
    `calls` back-to-back calls, eager and replayed from a HIP graph that
    captured one call (the plan is resident, so the call only launches)."""
    import torch
    lmax = 256
    g = sht.GeomHandle(si.gauss_legendre(lmax + 1, 2 * lmax + 1))
    a = torch.from_numpy(si.powerlaw_alm(lmax, lmax, si.config_seed(1))).cuda()
    out = torch.zeros(g.npix, dtype=torch.float64, device="cuda")
    ws = sht.workspace(lmax, lmax, g, 1, "cuda")
    sht.prepare(g, lmax)
    for _ in range(10):
        sht.alm2map(a, g, lmax, out=out, ws=ws)
    torch.cuda.synchronize()
    ref = out.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        for _ in range(calls):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / calls, (time.perf_counter() - t0) * 1e6 / calls

    eager_us, eager_host_us = timed(lambda: sht.alm2map(a, g, lmax, out=out, ws=ws))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        sht.alm2map(a, g, lmax, out=out, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sht.alm2map(a, g, lmax, out=out, ws=ws)
    out.zero_()
    graph.replay()
    torch.cuda.synchronize()
    if not torch.equal(out, ref):
        raise RuntimeError("graph replay differs from the eager call")
    graph_us, graph_host_us = timed(graph.replay)
    return {"workload": "FP64 alm2map, Gauss-Legendre 257 x 513, lmax=mmax=256, 1 map", "calls": calls,
            "eager_us_per_map": eager_us, "graph_us_per_map": graph_us,
            "eager_host_us_per_call": eager_host_us, "graph_host_us_per_call": graph_host_us}


def config4(sht, si, steps, warmup, nreq=256):
    """The uneven batch: nreq single-map requests, lmax = round(exp U[ln 128,
    ln 2048]), each on its own Gauss-Legendre grid of (lmax+1) x (2 lmax+1)
    points, alm2map or map2alm with equal odds; map2alm inputs are FP64
    alm2map outputs of power-law a_lm, so (exact quadrature) every map2alm
    must return its seed a_lm.  Timed three ways on one stream: the batch
    (sht_batch_run: ring analysis, one persistent Legendre launch for every
    request, ring synthesis) replayed from a HIP graph; and the per-request
    loop of sht_alm2map / sht_map2alm calls, FP64 and mixed precision."""
    import numpy as np
    import torch
    rng = np.random.default_rng(si.config_seed(4))
    lms = np.round(np.exp(rng.uniform(np.log(128), np.log(2048), nreq))).astype(int)
    kinds = np.where(rng.random(nreq) < 0.5, "alm2map", "map2alm")
    t0 = time.perf_counter()
    geoms = [sht.GeomHandle(si.gauss_legendre(L + 1, 2 * L + 1)) for L in lms.tolist()]
    seeds, inputs = [], []
    for i, (L, k, gh) in enumerate(zip(lms.tolist(), kinds.tolist(), geoms)):
        a = torch.from_numpy(si.powerlaw_alm(L, L, si.config_seed(4, i))).cuda()
        seeds.append(a)
        inputs.append(a if k == "alm2map" else sht.alm2map(a, gh, L))
    torch.cuda.synchronize()
    batch = sht.Batch([(k, L, gh, x, None) for k, L, gh, x in zip(kinds.tolist(), lms.tolist(), geoms, inputs)],
                      tiles="auto")
    setup_s = time.perf_counter() - t0
    print(f"[config4] {nreq} requests, plans and batch built in {setup_s:.1f} s", file=sys.stderr, flush=True)
    for _ in range(warmup):
        batch.run()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(n):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return times

    t_graph = timed(graph.replay, steps)
    t_eager = timed(batch.run, steps)
    # per-request loop, buffers preallocated
    outs = [torch.empty_like(o) for o in batch.outputs]
    wss = {f: [sht.workspace(L, L, gh, 1, "cuda", f) for L, gh in zip(lms.tolist(), geoms)] for f in (0, sht.SHT_MIXED)}

    def loop(flags):
        def run():
            for i, (k, L, gh, x) in enumerate(zip(kinds.tolist(), lms.tolist(), geoms, inputs)):
                fn = sht.alm2map if k == "alm2map" else sht.map2alm
                fn(x, gh, L, out=outs[i], ws=wss[flags][i], flags=flags)
        return run

    t_loop = timed(loop(0), max(2, steps // 2))
    loop_out = [o.clone() for o in outs]
    t_loop_mx = timed(loop(sht.SHT_MIXED), max(2, steps // 2))
    rel = lambda x, y: (x - y).norm().item() / y.norm().item()
    ana = [i for i, k in enumerate(kinds.tolist()) if k == "map2alm"]
    syn = [i for i, k in enumerate(kinds.tolist()) if k == "alm2map"]
    err_ana = max(rel(batch.outputs[i], seeds[i]) for i in ana)
    err_syn = max(rel(batch.outputs[i], loop_out[i]) for i in syn)
    err_mx_ana = max(rel(outs[i], seeds[i]) for i in ana)
    nslots = [(L + 2) // 2 for L in lms.tolist()]
    flops = sum(FLOPS_PER_TRIPLE * ns * (L + 1) * (L + 2) // 2 for ns, L in zip(nslots, lms.tolist()))
    ms = float(np.median(t_graph))
    batch.close()
    return {
        "workload": (f"uneven batch: {nreq} single-map requests, lmax log-uniform in [128, 2048] on their own "
                     f"Gauss-Legendre grids, {len(syn)} alm2map + {len(ana)} map2alm, FP64"),
        "value": nreq * 1000.0 / ms, "unit": "maps/s", "ms_per_batch": ms,
        "latency_ms": latency(t_graph),
        "eager_ms_per_batch": float(np.median(t_eager)),
        "per_request_loop_fp64": {"ms_per_batch": float(np.median(t_loop)),
                                  "value": nreq * 1000.0 / float(np.median(t_loop))},
        "per_request_loop_mixed": {"ms_per_batch": float(np.median(t_loop_mx)),
                                   "value": nreq * 1000.0 / float(np.median(t_loop_mx)),
                                   "map2alm_relrms_vs_seed_max": err_mx_ana},
        "speedup_vs_per_request_fp64": float(np.median(t_loop)) / ms,
        "legendre_flops_per_batch": flops,
        "legendre_tflops_whole_batch": flops / (ms * 1e-3) / 1e12,
        "errors": {"map2alm_relrms_vs_seed_max": err_ana, "alm2map_relrms_vs_single_calls_max": err_syn},
        "lmax_range": [int(lms.min()), int(lms.max())], "setup_s": setup_s,
    }


def copy_probe(nbytes: int) -> None:
    """A plain device copy of known size, for calibrating HBM byte counters."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nside", type=int, default=1024)
    ap.add_argument("--lmax", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=64,
                    help="maps in the batched mixed-precision alm2map leg (0: skip it)")
    ap.add_argument("--serve", type=int, default=256,
                    help="requests in the serving leg (mixed lmax in [64, 4096]; 0: skip it)")
    ap.add_argument("--serve-slots", type=int, default=4, help="concurrent requests (HIP streams) in the serving leg")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0, help="HBM budget of the serving leg")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--no-config4", action="store_true",
                    help="skip the uneven-batch leg (256 requests, lmax 128..2048, one persistent Legendre launch)")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the batched Gauss-Legendre leg (1025 x 2049, lmax 1024, 64 maps)")
    ap.add_argument("--no-small-latency", action="store_true",
                    help="skip the launch-bound lmax=256 latency leg (e.g. to profile the main step alone)")
    ap.add_argument("--copy-probe", type=int, default=0, help="run only a device copy of this many bytes")
    ap.add_argument("--peak-probe", action="store_true",
                    help="run only the throughput probes (FP64 FMA, FP32 and BF16 matrix instructions, and "
                         "whether FP32 matrix and FP64 vector work overlap)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); run it with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.peak_probe:
        from paper_1106_0159_amd import probe
        rates = [probe.rate(k) for k in probe.KINDS if k != "fp32_mfma_with_fp64_fma"]
        print(json.dumps({"peak_probe": rates, "coexec": probe.coexec(),
                          "nominal_tflops": {"fp64_fma": PEAK_FP64_VALU_TFLOPS,
                                             "fp32_mfma_16x16x4": PEAK_FP32_MFMA_TFLOPS,
                                             "bf16_mfma_16x16x32": 2500.0}}))
        return

    import numpy as np
    import torch

    import paper_1106_0159_amd as sht
    import sht_inputs as si

    if args.serve_only:
        torch.cuda.set_device(0)
        print(json.dumps({"serving": serving(sht, si, max(1, args.serve), args.serve_slots, args.serve_budget_gb)}),
              flush=True)
        return

    nside = args.nside
    lmax = args.lmax if args.lmax is not None else 2 * nside
    g = si.healpix(nside)
    gh = sht.GeomHandle(g)
    a_np = si.powerlaw_alm(lmax, lmax, si.config_seed(2))
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    a = torch.from_numpy(a_np).to(dev)
    delta = torch.empty((g.nrings, lmax + 1), dtype=torch.complex128, device=dev)
    delta_s = torch.empty_like(delta)
    mp = torch.zeros(g.npix, dtype=torch.float64, device=dev)
    a_out = torch.empty_like(a)
    ws = sht.workspace(lmax, lmax, gh, 1, dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        sht.alm2delta(a, gh, lmax, lmax, out=delta, ws=ws)
        if ev is not None:
            ev[1].record()
        sht.delta2map(delta, gh, lmax, out=mp)
        if ev is not None:
            ev[2].record()
        sht.map2delta(mp, gh, lmax, out=delta_s)
        if ev is not None:
            ev[3].record()
        sht.delta2alm(delta_s, gh, lmax, lmax, out=a_out, ws=ws)
        if ev is not None:
            ev[4].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_names = ["leg_syn", "fft_syn", "fft_ana", "leg_ana"]
    stage_ms = {n: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(K)]))
                for i, n in enumerate(stage_names)}
    step_times = np.array([evs[k][0].elapsed_time(evs[k][4]) for k in range(K)])
    step_ms = float(np.mean(step_times))
    ms_per_step = max(wall * 1000.0 / K, step_ms)

    nslots = mirror_slots(g.theta)
    triples = count_triples(nslots, lmax, lmax)
    flops = FLOPS_PER_TRIPLE * triples
    dom = max(("leg_syn", "leg_ana"), key=lambda n: stage_ms[n])
    achieved = flops / (stage_ms[dom] * 1e-3) / 1e12
    counters = stored_counters(dom)
    executed = counters.get("fp64_flops_per_launch")
    rec = {
        "metric": "maps/s at lmax=2048 (plain FP64 vs batched mixed); p50/p99 solve latency",
        "value": 1000.0 / ms_per_step,
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"FP64 alm2map+map2alm, HEALPix nside={nside}, lmax=mmax={lmax}, 1 map, power-law a_lm",
            "mode": "plain_fp64",
            "nside": nside, "lmax": lmax, "mmax": lmax, "nmaps": 1,
            "nrings": g.nrings, "npix": g.npix, "slots": nslots,
        },
        "stages_ms": stage_ms,
        "latency_ms": latency(step_times),
        "fft_roofline": fft_roofline(g, lmax, 1, stage_ms),
        "alm2map_maps_per_s": 1000.0 / (stage_ms["leg_syn"] + stage_ms["fft_syn"]),
        "map2alm_maps_per_s": 1000.0 / (stage_ms["fft_ana"] + stage_ms["leg_ana"]),
        "roofline": {
            "kernel": {"leg_syn": "k_prescale + k_leg_syn",
                       "leg_ana": "k_leg_ana (+ k_ana_combine above 2048 slots)"}[dom],
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VALU_TFLOPS,
            "traffic": counters.get("bytes_per_launch"),
            "flops_per_launch": flops,
            "executed_fp64_flops_per_launch": executed,
            "executed_tflops": None if executed is None else executed / (stage_ms[dom] * 1e-3) / 1e12,
        },
    }
    if args.batch > 0:
        rec["batched_mixed"], rec["batched_fp64"] = batched_legs(sht, si, gh, g, lmax, args.batch, max(3, K // 4),
                                                                 args.warmup, nslots, mp, a_out)
        print(f"[batch] mixed {rec['batched_mixed']['value']:.0f} maps/s, "
              f"fp64 {rec['batched_fp64']['value']:.0f} maps/s", file=sys.stderr, flush=True)
    if not args.no_config3:
        rec["config3"] = config3(sht, si, max(3, K // 4), args.warmup, not args.no_cpu_baseline)
        print(f"[config3] mixed {rec['config3']['mixed']['value']:.0f} maps/s, "
              f"fp64 {rec['config3']['fp64']['value']:.0f} maps/s", file=sys.stderr, flush=True)
    if not args.no_config4:
        rec["config4"] = config4(sht, si, max(5, K // 2), args.warmup)
        print(f"[config4] batch {rec['config4']['value']:.0f} maps/s ({rec['config4']['ms_per_batch']:.2f} ms), "
              f"per-request loop {rec['config4']['per_request_loop_fp64']['value']:.0f} maps/s", file=sys.stderr,
              flush=True)
    if not args.no_small_latency:
        rec["small_latency"] = small_latency(sht, si)
        print(f"[small] eager {rec['small_latency']['eager_us_per_map']:.1f} us/map, "
              f"graph {rec['small_latency']['graph_us_per_map']:.1f} us/map", file=sys.stderr, flush=True)
    if args.serve > 0:
        rec["serving"] = serving(sht, si, args.serve, args.serve_slots, args.serve_budget_gb)
    if not args.no_cpu_baseline:
        mp_np = mp.cpu().numpy()
        rec["cpu_baseline"] = cpu_baseline(g, lmax, a_np, mp_np)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
