"""Benchmark: FP64 alm2map + map2alm on HEALPix N_side=1024, lmax=mmax=2048.

One step = one map through both transforms, with inputs resident in HBM:
    alm --(Legendre synthesis)--> Delta --(ring FFT synthesis)--> map
    map --(ring FFT analysis)--> Delta^S --(Legendre analysis)--> alm'
called through the four stage entry points of the C ABI (their composition is
exactly sht_alm2map followed by sht_map2alm), with HIP events on the launch
stream between stages.  A second leg ("batched_mixed" in the output) runs
the same two transforms on a batch of 64 maps with the mixed-precision
Legendre contraction.
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
    """Number of ring slots (mirror pairs plus unpaired rings), as the library forms them."""
    th = sorted(float(t) for t in theta)
    i, j, n = 0, len(th) - 1, 0
    while i <= j:
        if i == j:
            n += 1
            break
        d = th[i] + th[j] - math.pi
        if abs(d) <= 1e-14:
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


def batched_mixed(sht, si, gh, g, lmax, nmaps, steps, warmup, nslots, mp_fp64, a_fp64):
    """One batch of power-law maps through both transforms with SHT_MIXED
    (FP64 recurrence, FP32 matrix-core contraction; Delta and FFTs FP64,
    Delta map-minor in synthesis), through the four stage entry points, HIP events on
    the launch stream around each stage.  Map 0 of the batch is the map of the
    plain FP64 step: the relative RMS differences of its map and of its
    analysed a_lm to the FP64 results are reported."""
    import numpy as np
    import torch
    dev = torch.device("cuda", 0)
    alm = torch.empty((nmaps, si.nalm(lmax, lmax)), dtype=torch.complex128, device=dev)
    for i in range(nmaps):
        alm[i] = torch.from_numpy(si.powerlaw_alm(lmax, lmax, si.config_seed(2, i))).to(dev)
    # Delta as sht_alm2map / sht_map2alm keep it with SHT_MIXED (the stage
    # calls give the same bits as the combined ones): map-minor,
    # [nrings][mmax+1][nmaps], in synthesis and ring-major in analysis
    delta = torch.empty((g.nrings, lmax + 1, nmaps), dtype=torch.complex128, device=dev)
    delta_s = torch.empty((nmaps, g.nrings, lmax + 1), dtype=torch.complex128, device=dev)
    mp = torch.zeros((nmaps, g.npix), dtype=torch.float64, device=dev)
    a_out = torch.empty_like(alm)
    ws = sht.workspace(lmax, lmax, gh, nmaps, dev, sht.SHT_MIXED)
    MM = sht.SHT_DELTA_MAP_MINOR
    F = sht.SHT_MIXED | MM

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        sht.alm2delta(alm, gh, lmax, lmax, out=delta, ws=ws, flags=F)
        mark(1)
        sht.delta2map(delta, gh, lmax, out=mp, flags=MM)
        mark(2)
        sht.map2delta(mp, gh, lmax, out=delta_s)
        mark(3)
        sht.delta2alm(delta_s, gh, lmax, lmax, out=a_out, ws=ws, flags=sht.SHT_MIXED)
        mark(4)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    names = ["leg_syn_mx", "fft_syn", "fft_ana", "leg_ana_mx"]
    st = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs])) for i, n in enumerate(names)}
    batch_times = np.array([e[0].elapsed_time(e[4]) for e in evs])
    ms = max(wall * 1000.0 / steps, sum(st.values()))
    flops = 4 * nmaps * count_triples(nslots, lmax, lmax)  # matrix-core flops of one contraction
    dom = max(("leg_syn_mx", "leg_ana_mx"), key=lambda n: st[n])
    achieved = flops / (st[dom] * 1e-3) / 1e12
    rel = lambda x, y: (x - y).norm().item() / y.norm().item()
    return {
        "direction": "alm2map+map2alm",
        "nmaps": nmaps,
        "value": nmaps * 1000.0 / ms,
        "unit": "maps/s",
        "ms_per_batch": ms,
        "latency_ms": latency(batch_times),
        "steps": steps,
        "stages_ms": st,
        "alm2map_maps_per_s": nmaps * 1000.0 / (st["leg_syn_mx"] + st["fft_syn"]),
        "map2alm_maps_per_s": nmaps * 1000.0 / (st["fft_ana"] + st["leg_ana_mx"]),
        "dtype": "f64 recurrence, f32 contraction",
        "relrms_map0_vs_fp64": rel(mp[0], mp_fp64),
        "relrms_alm0_vs_fp64": rel(a_out[0], a_fp64),
        "roofline": {
            "kernel": {"leg_syn_mx": "k_prescale_mx + k_leg_syn_mx",
                       "leg_ana_mx": "k_leg_ana_mx"}[dom],
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_FP32_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
            "traffic": None,
            "flops_per_launch": flops,
        },
    }


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
    ap.add_argument("--no-small-latency", action="store_true",
                    help="skip the launch-bound lmax=256 latency leg (e.g. to profile the main step alone)")
    ap.add_argument("--copy-probe", type=int, default=0, help="run only a device copy of this many bytes")
    ap.add_argument("--peak-probe", action="store_true",
                    help="run only the throughput probes (FP64 FMA, FP32 and BF16 matrix instructions)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); run it with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.peak_probe:
        import paper_1106_0159_amd as sht
        rates = [sht.probe_rate(k) for k in sht.PROBE_KINDS]
        print(json.dumps({"peak_probe": rates,
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
        rec["batched_mixed"] = batched_mixed(sht, si, gh, g, lmax, args.batch, max(3, K // 4), args.warmup,
                                             nslots, mp, a_out)
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
