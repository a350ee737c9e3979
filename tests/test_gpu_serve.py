"""GPU tests of the continuous-batching server (paper_1106_0159_amd.serve).

A mix of alm2map and map2alm requests on HEALPix and Gauss-Legendre grids of
different lmax runs through the server.  It is checked that:
- each result is bitwise the same alone and in the mix, in both precision
  modes (each request runs on its own stream and the kernels are
  deterministic);
- admission keeps the bytes in flight within the HBM budget while several
  requests overlap;
- a request larger than the budget is rejected;
- plans evicted while other requests are in flight do not change any result;
- an uneven batch, each request on its own Gauss-Legendre grid, returns the
  seed a_lm from map2alm of FP64 maps (exact quadrature).
One request of each kind is also held to the oracle (relative RMS <= 1e-12
in FP64, <= 1e-6 in mixed precision).
"""
import sys

import numpy as np
import pytest

import oracle
import sht_inputs as si

pytestmark = pytest.mark.gpu

# (kind, lmax, grid, nmaps)
SPECS = [
    ("alm2map", 16, "hp", 1), ("map2alm", 24, "hp", 1), ("alm2map", 64, "gl", 1), ("map2alm", 40, "hp", 1),
    ("alm2map", 96, "hp", 1), ("map2alm", 64, "gl", 1), ("alm2map", 30, "gl", 3), ("map2alm", 128, "hp", 1),
    ("alm2map", 128, "hp", 1), ("map2alm", 16, "hp", 2), ("alm2map", 48, "hp", 1), ("map2alm", 96, "gl", 1),
]


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_1106_0159_amd as sht
    from paper_1106_0159_amd import serve
    sht.lib()
    grids, inputs = {}, []
    for i, (kind, L, gk, nm) in enumerate(SPECS):
        key = (gk, L)
        if key not in grids:
            g = si.healpix(L // 2) if gk == "hp" else si.gauss_legendre(L + 1, 2 * L + 1)
            grids[key] = (g, sht.GeomHandle(g))
        g = grids[key][0]
        if kind == "alm2map":
            x = np.stack([si.powerlaw_alm(L, L, si.config_seed(5, 100 * i + j)) for j in range(nm)])
        else:
            x = np.stack([si.random_map(g, si.config_seed(5, 100 * i + j)) for j in range(nm)])
        inputs.append((x, torch.from_numpy(x).cuda()))
    return sht, serve, grids, inputs


def requests(env, arrivals=None):
    sht, serve, grids, inputs = env
    return [serve.Request(kind, L, grids[(gk, L)][1], inputs[i][1],
                          arrival=None if arrivals is None else float(arrivals[i]))
            for i, (kind, L, gk, nm) in enumerate(SPECS)]


def alone(env, flags):
    sht, serve, grids, inputs = env
    out = []
    for r in requests(env):
        srv = serve.Server(64 << 30, 1, flags)
        assert srv.submit(r)
        srv.drain()
        assert r.status == "done", r.error
        out.append(r.result.clone())
    return out


def bitwise_same(reqs, ref):
    import torch
    torch.cuda.synchronize()
    for r, a in zip(reqs, ref):
        assert r.status == "done", (r.rid, r.status, r.error)
        assert torch.equal(r.result, a), f"request {r.rid} ({r.kind} lmax={r.lmax}) differs from its solo run"


@pytest.mark.parametrize("flags", [0, 1], ids=["fp64", "mixed"])
def test_same_alone_and_in_the_mix(env, flags):
    sht, serve, grids, inputs = env
    say(f"serve mix flags={flags}: solo runs")
    ref = alone(env, flags)
    reqs = requests(env)
    needs = [serve.request_bytes(r.kind, r.lmax, r.lmax, r.geom, r.nmaps, flags)[0] for r in reqs]
    budget = int(2.5 * max(needs))  # the largest requests wait for room, the small ones overlap
    say(f"serve mix flags={flags}: {len(reqs)} requests, budget {budget} B, 4 slots")
    srv = serve.Server(budget, 4, flags)
    for r in reqs:
        assert srv.submit(r)
    srv.drain()
    st = srv.stats()
    assert st["done"] == len(reqs) and st["rejected"] == 0
    assert srv.adm.max_used <= budget and srv.adm.used == 0
    assert srv.adm.max_running >= 2, "no two requests were ever in flight together"
    bitwise_same(reqs, ref)
    # one request of each kind against the oracle
    tol = 1e-12 if flags == 0 else 1e-6
    for i in (0, 1):
        kind, L, gk, nm = SPECS[i]
        g = grids[(gk, L)][0]
        x = inputs[i][0][0]
        want = oracle.alm2map(L, L, g, x) if kind == "alm2map" else oracle.map2alm(L, L, g, x)
        got = reqs[i].result.cpu().numpy().reshape(-1)
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        say(f"serve oracle {kind} lmax={L}: rel rms {err:.2e}")
        assert err <= tol, (kind, L, err)


def test_poisson_arrivals(env):
    import torch
    sht, serve, grids, inputs = env
    ref = alone(env, 0)
    rng = np.random.default_rng(si.config_seed(5, 9999))
    arr = np.cumsum(rng.exponential(1.0 / 3000.0, len(SPECS)))
    arr -= arr[0]
    say(f"serve Poisson trace: {len(SPECS)} requests over {arr[-1] * 1e3:.2f} ms")
    reqs = requests(env, arr)
    srv = serve.Server(64 << 30, 4, 0)
    srv.run_trace(reqs)
    st = srv.stats()
    assert st["done"] == len(reqs)
    lat = [r.latency for r in reqs]
    assert min(lat) > 0 and st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert all(r.t_admit >= r.arrival for r in reqs)
    # first come, first served: admission times follow arrival order
    order = sorted(reqs, key=lambda r: r.arrival)
    assert all(a.t_admit <= b.t_admit for a, b in zip(order, order[1:]))
    bitwise_same(reqs, ref)
    torch.cuda.synchronize()


def test_over_budget_request_is_rejected(env):
    sht, serve, grids, inputs = env
    reqs = requests(env)
    big = max(reqs, key=lambda r: serve.request_bytes(r.kind, r.lmax, r.lmax, r.geom, r.nmaps)[0])
    need = serve.request_bytes(big.kind, big.lmax, big.lmax, big.geom, big.nmaps)[0]
    srv = serve.Server(need - 1, 2, 0)
    say(f"serve reject: need {need} B over budget {need - 1} B")
    assert not srv.submit(big)
    assert big.status == "rejected" and big.result is None
    assert srv.poll() == 0 and srv.adm.used == 0


def test_plan_eviction_while_in_flight(env):
    sht, serve, grids, inputs = env
    ref = alone(env, 0)
    say("serve with plan cache limits (1, 1): every new grid evicts the last")
    try:
        sht.plan_cache_limits(1, 1)
        reqs = requests(env)
        srv = serve.Server(64 << 30, 4, 0)
        for r in reqs:
            srv.submit(r)
        srv.drain()
        bitwise_same(reqs, ref)
    finally:
        sht.plan_cache_limits(8, 32)


def test_prepare_keeps_plans_resident(env):
    sht, serve, grids, inputs = env
    sht.plan_cache_limits(64, 64)
    try:
        for (gk, L), (g, gh) in grids.items():
            sht.prepare(gh, L)
        held = sht.plan_cache_bytes()
        say(f"serve prepare: {len(grids)} grids, plan cache {held} B")
        assert held > 0
        for (gk, L), (g, gh) in grids.items():
            sht.prepare(gh, L)  # all resident: nothing new is built
        assert sht.plan_cache_bytes() == held
    finally:
        sht.plan_cache_limits(8, 32)


@pytest.mark.parametrize("flags", [0, 1], ids=["fp64", "mixed"])
def test_uneven_gauss_legendre_batch(env, flags):
    """The uneven batch: each request on its own Gauss-Legendre grid of
    (lmax+1) x (2 lmax+1) points, lmax log-uniform, alm2map or map2alm with
    equal odds.  The map2alm inputs are FP64 alm2map outputs of seeded a_lm,
    and Gauss-Legendre quadrature is exact at this band limit, so every
    map2alm result is the seed a_lm (to 1e-12 in FP64, 1e-6 mixed); every
    alm2map result matches the FP64 transform (bitwise in FP64, 1e-6 mixed)."""
    import torch
    sht, serve, grids, inputs = env
    rng = np.random.default_rng(si.config_seed(4))
    n = 12
    lms = np.round(np.exp(rng.uniform(np.log(16), np.log(96), n))).astype(int)
    kinds = np.where(rng.random(n) < 0.5, "alm2map", "map2alm")
    say(f"uneven GL batch flags={flags}: lmax {lms.tolist()}")
    reqs, want = [], []
    for i, (L, k) in enumerate(zip(lms.tolist(), kinds.tolist())):
        gh = sht.GeomHandle(si.gauss_legendre(L + 1, 2 * L + 1))
        a = torch.from_numpy(si.powerlaw_alm(L, L, si.config_seed(4, i))).cuda()
        m64 = sht.alm2map(a, gh, L)
        reqs.append(serve.Request(k, L, gh, a if k == "alm2map" else m64))
        want.append(m64 if k == "alm2map" else a)
    srv = serve.Server(64 << 30, 4, flags)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    torch.cuda.synchronize()
    for r, w in zip(reqs, want):
        assert r.status == "done", r.error
        got = r.result.reshape(w.shape)
        err = ((got - w).norm() / w.norm()).item()
        tol = (0.0 if r.kind == "alm2map" else 1e-12) if flags == 0 else 1e-6
        assert err <= tol, (r.kind, r.lmax, err)


def test_pinned_plan_is_not_evicted(env):
    """sht_prepare(..., SHT_PIN) keeps a plan resident through LRU eviction
    at cache limits of 1 (the cache grows past its limit instead); once
    unpinned it is evicted like any other.  Residency is read through
    sht_plan_cache_bytes: preparing a resident plan builds nothing."""
    sht, serve, grids, inputs = env
    g1, L1 = si.healpix(8), 16
    gh1 = sht.GeomHandle(g1)
    others = [sht.GeomHandle(si.gauss_legendre(9, 17 + k)) for k in range(4)]
    say("pinned plan under cache limits of 1")
    sht.shutdown()
    try:
        sht.plan_cache_limits(1, 1)
        sht.prepare(gh1, L1, pin=True)
        for gh in others:
            sht.prepare(gh, 8)  # each evicts the previous unpinned plan, never the pinned one
        held = sht.plan_cache_bytes()
        sht.prepare(gh1, L1)  # resident: nothing is built
        assert sht.plan_cache_bytes() == held
        a = si.powerlaw_alm(L1, L1, 3)
        import torch
        got = sht.alm2map(torch.from_numpy(a).cuda(), gh1, L1)
        torch.cuda.synchronize()
        ref = oracle.alm2map(L1, L1, g1, a)
        assert np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-12
        sht.unpin(gh1, L1)
        sht.plan_cache_limits(1, 1)  # now the unpinned extras go
        assert sht.plan_cache_bytes() < held
        with pytest.raises(sht.ShtError) as e:
            sht.unpin(gh1, L1)
        assert e.value.code == sht.SHT_ENOPLAN
    finally:
        sht.plan_cache_limits(8, 32)


def test_injected_allocation_failure_leaves_no_leak_and_no_partial_plan(env):
    """Every plan-table allocation of a fresh build in turn fails (the
    library's SHT_TEST_FAIL_ALLOC test hook): the build returns SHT_ENOMEM,
    the cache keeps only complete entries and loses no bytes (after a
    shutdown the plan bytes are 0 again), and a build without the failure
    then gives the same cache size as a clean one and correct results."""
    import os
    import torch
    sht, serve, grids, inputs = env
    L, g = 24, si.healpix(8)
    gh = sht.GeomHandle(g)
    a = si.powerlaw_alm(L, L, 31)
    ref = oracle.alm2map(L, L, g, a)
    sht.shutdown()
    assert sht.plan_cache_bytes() == 0
    sht.prepare(gh, L)
    clean = sht.plan_cache_bytes()
    say(f"allocation failure injection: clean plan {clean} bytes")
    k, failures = 1, 0
    try:
        while k < 200:
            sht.shutdown()
            assert sht.plan_cache_bytes() == 0, k  # nothing leaked by the last attempt
            os.environ["SHT_TEST_FAIL_ALLOC"] = str(k)
            try:
                sht.prepare(gh, L)
                ok = True
            except sht.ShtError as e:
                assert e.code == sht.SHT_ENOMEM, (k, e.code)
                ok = False
            del os.environ["SHT_TEST_FAIL_ALLOC"]
            if ok:
                break
            failures += 1
            assert sht.plan_cache_bytes() <= clean, k  # only complete entries stay
            sht.prepare(gh, L)
            assert sht.plan_cache_bytes() == clean, k
            got = sht.alm2map(torch.from_numpy(a).cuda(), gh, L)
            torch.cuda.synchronize()
            assert np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-12, k
            k += 1
    finally:
        os.environ.pop("SHT_TEST_FAIL_ALLOC", None)
    say(f"allocation failure injection: {failures} failing allocations checked")
    assert failures >= 10  # coefficient, geometry, FFT and start tables all took their turn
