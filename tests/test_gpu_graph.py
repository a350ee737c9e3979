"""Transforms captured in HIP graphs.

Once a grid's plan is resident (sht_prepare), a transform call enqueues only
kernels and the events that fork and join the ring-FFT side streams: no
allocation, copy, memset or synchronisation.  It can then be captured in a
HIP graph and replayed.  Each replay here is checked bitwise against the eager
result, with eager work on other buffers and synchronisations between
replays."""
import sys

import numpy as np
import pytest

import sht_inputs as si

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("flags", [0, 1, 17], ids=["fp64", "mixed", "mixed-split-bf16"])
@pytest.mark.parametrize("grid", ["gl", "hp"])
def test_graph_replays_equal_eager(grid, flags):
    import torch
    import paper_1106_0159_amd as sht
    lmax = 64 if grid == "hp" else 48
    g = sht.GeomHandle(si.healpix(32) if grid == "hp" else si.gauss_legendre(lmax + 1, 2 * lmax + 1))
    nm = 8 if flags else 1
    fa = flags & ~sht.SHT_MIXED_SPLIT_BF16  # a synthesis variant: analysis takes the FP32 products
    say(f"graph {grid} lmax={lmax} flags={flags} nmaps={nm}")
    a = torch.from_numpy(np.stack([si.powerlaw_alm(lmax, lmax, si.config_seed(1, i)) for i in range(nm)])).cuda()
    sht.prepare(g, lmax, flags=flags)
    mp = torch.zeros((nm, g.npix), dtype=torch.float64, device="cuda")
    back = torch.empty_like(a)
    ws = sht.workspace(lmax, lmax, g, nm, "cuda", flags)
    sht.alm2map(a, g, lmax, out=mp, ws=ws, flags=flags)
    sht.map2alm(mp, g, lmax, out=back, ws=ws, flags=fa)
    torch.cuda.synchronize()
    mp_ref, back_ref = mp.clone(), back.clone()
    # warm the capture stream, then capture one round trip
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        sht.alm2map(a, g, lmax, out=mp, ws=ws, flags=flags)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sht.alm2map(a, g, lmax, out=mp, ws=ws, flags=flags)
        sht.map2alm(mp, g, lmax, out=back, ws=ws, flags=fa)
    other = torch.from_numpy(si.powerlaw_alm(lmax, lmax, 99)).cuda()
    for rep in range(4):
        mp.zero_()
        back.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(mp, mp_ref), f"replay {rep}: map differs"
        assert torch.equal(back, back_ref), f"replay {rep}: a_lm differs"
        # eager work between replays, on other buffers
        sht.alm2map(other, g, lmax)
        torch.cuda.synchronize()
