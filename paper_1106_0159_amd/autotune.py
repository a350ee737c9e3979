"""Tile autotuner for uneven batches (sht_batch_*).

The persistent Legendre kernel takes its work in tiles whose shape is chosen
per request (sht_request.tile = 16 * shape + T):
  synthesis  shape 0: one wave per (m, 64 T ring slots), T in {1, 2, 4};
  analysis   shape 0: one wave per m holding every slot (64 T >= slots), or
             shape 1: one workgroup per (m, group of 256 T slots), T in {1, 2, 4}.
The best shape depends on lmax and on the number of ring slots (mirror ring
pairs plus unpaired rings).  tune() times every admissible shape on a small
batch of Gauss-Legendre requests per (lmax bucket, slot bucket), keeps the
fastest, and writes the table as JSON; choose() looks a request up in it.
The library's own default is used for buckets that the table lacks.

    python -m paper_1106_0159_amd.autotune [--out tiles.json] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles.json")
# bucket edges (upper bounds, inclusive) for lmax and for the ring-slot count
LMAX_EDGES = (64, 128, 256, 512, 1024, 2048, 4096)
SLOT_EDGES = (64, 128, 256, 512, 1024, 2048, 4096)


def bucket(lmax: int, nslots: int) -> str:
    bl = next((e for e in LMAX_EDGES if lmax <= e), LMAX_EDGES[-1])
    bs = next((e for e in SLOT_EDGES if nslots <= e), SLOT_EDGES[-1])
    return f"l{bl}_s{bs}"


def candidates(kind: str, nslots: int):
    if kind == "alm2map":
        return [1, 2, 4]
    out = [t for t in (1, 2, 4) if 64 * t >= nslots]
    return out + [16 + t for t in (1, 2, 4)]


def gl_slots(nrings: int) -> int:
    """Ring slots of a Gauss-Legendre grid: mirror pairs plus the equator ring."""
    return (nrings + 1) // 2


def load(path: str = TABLE_PATH) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def choose(table: dict, kind: str, lmax: int, nslots: int) -> int:
    """The tuned tile code for a request, or 0 (the library's choice)."""
    t = table.get(kind, {}).get(bucket(lmax, nslots))
    if t is None or t not in candidates(kind, nslots):
        return 0
    return int(t)


def _time_batch(sht, reqs, reps: int) -> float:
    import torch
    b = sht.Batch(reqs)
    b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = math.inf
    for _ in range(reps):
        e0.record()
        b.run()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    b.close()
    return best


def tune(reps: int = 5, per_bucket: int = 6, lmaxes=(48, 96, 192, 384, 768, 1536), verbose: bool = True) -> dict:
    """Times every admissible tile on `per_bucket` requests of each kind at
    each lmax (Gauss-Legendre grids of (lmax+1) x (2 lmax+1) points, lmax
    spread over the bucket) and returns the table."""
    import numpy as np
    import torch

    import paper_1106_0159_amd as sht
    import sht_inputs as si
    table = {"alm2map": {}, "map2alm": {}, "timings_ms": {}, "device": torch.cuda.get_device_name(0),
             "reps": reps, "per_bucket": per_bucket, "written": time.strftime("%Y-%m-%d %H:%M:%S")}
    for L0 in lmaxes:
        Ls = [max(2, int(round(L0 * f))) for f in np.linspace(0.8, 1.2, per_bucket)]
        grids = [si.gauss_legendre(L + 1, 2 * L + 1) for L in Ls]
        ns = gl_slots(Ls[0] + 1)
        for kind in ("alm2map", "map2alm"):
            xs = [torch.from_numpy(si.powerlaw_alm(L, L, 7 + i)).cuda() if kind == "alm2map"
                  else torch.from_numpy(si.random_map(g, 7 + i)).cuda() for i, (L, g) in enumerate(zip(Ls, grids))]
            key = bucket(Ls[0], ns)
            res = {}
            for t in candidates(kind, max(gl_slots(L + 1) for L in Ls)):
                res[t] = _time_batch(sht, [(kind, L, g, x, None, t) for L, g, x in zip(Ls, grids, xs)], reps)
            best = min(res, key=res.get)
            table[kind][key] = best
            table["timings_ms"][f"{kind}:{key}"] = {str(k): round(v, 4) for k, v in res.items()}
            if verbose:
                print(f"[autotune] {kind} {key} (lmax ~{L0}): " +
                      ", ".join(f"{k}: {v:.3f} ms" for k, v in res.items()) + f" -> {best}", flush=True)
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    table = tune(args.reps)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"[autotune] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
