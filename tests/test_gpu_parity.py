"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar: relative RMS <= 1e-12 for FP64 results (maps, a_lm and Delta), on the
same seeded inputs.  Small cases compare every element; the full-size
HEALPix N_side=1024 / lmax=2048 case compares the whole synthesised map and
the whole analysed a_lm set; the Gauss-Legendre lmax=2048 grid compares every
fourth ring and every fourth m, aggregated.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import sht_inputs as si

import _oracle_cache as oc

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sht():
    import torch
    assert torch.cuda.is_available()
    import paper_1106_0159_amd as S
    S.lib()
    return S


def dev(x):
    import torch
    x = np.ascontiguousarray(x)
    return torch.from_numpy(x if x.flags.writeable else x.copy()).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relrms(got, ref):
    den = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / (den if den > 0 else 1.0)


def random_geometry(nr, seed, nphi_max=40):
    rng = np.random.default_rng(seed)
    th = np.sort(rng.uniform(0.0, math.pi, nr))
    nphi = rng.integers(1, nphi_max, nr).astype(np.int32)
    phi0 = rng.uniform(-3, 9, nr)
    w = rng.uniform(0.1, 1.0, nr)
    return si._pack(th, nphi, phi0, w, f"random{nr}")


SMALL_CASES = [
    # (name, geometry builder, lmax, mmax)
    ("gl0", lambda: si.gauss_legendre(1, 1), 0, 0),
    ("gl1", lambda: si.gauss_legendre(2, 3), 1, 1),
    ("gl2_odd", lambda: si.gauss_legendre(3, 5), 2, 2),
    ("gl3", lambda: si.gauss_legendre(4, 7), 3, 3),
    ("gl7_mless", lambda: si.gauss_legendre(8, 9), 7, 4),
    ("gl31", lambda: si.gauss_legendre(32, 63), 31, 31),
    ("gl64_odd", lambda: si.gauss_legendre(65, 129), 64, 64),
    ("hp4", lambda: si.healpix(4), 8, 8),
    ("hp8_alias", lambda: si.healpix(8), 40, 40),       # nphi = 4i < 2 mmax + 1 near the poles
    ("hp16", lambda: si.healpix(16), 32, 32),
    ("random_alias", lambda: random_geometry(23, 5), 30, 20),
    ("random_poles", lambda: si._pack(np.array([0.0, 0.4, 1.2, math.pi / 2, 2.0, math.pi]),
                                      np.array([1, 5, 16, 3, 9, 2], dtype=np.int32),
                                      np.array([0.0, 0.1, 2.0, -1.0, 0.5, 0.0]),
                                      np.ones(6), "poles"), 12, 12),
    ("gl_bluestein", lambda: si.gauss_legendre(70, 139), 69, 69),   # 139 is prime
    ("gl_radix13", lambda: si.gauss_legendre(40, 2 * 3 * 5 * 7 * 11 * 13 // 30), 39, 39),
    # more than 2048 unpaired rings: analysis needs two slot groups (partial a_lm
    # summed by the combine kernel); synthesis a ragged fifth tile
    ("random_many", lambda: random_geometry(2300, 11, nphi_max=12), 24, 24),
]


@pytest.mark.parametrize("case", SMALL_CASES, ids=[c[0] for c in SMALL_CASES])
def test_small_alm2map_and_map2alm(sht, case):
    name, mk, lmax, mmax = case
    g = mk()
    for kind, a in (("powerlaw", si.powerlaw_alm(lmax, mmax, 101)), ("uniform", si.uniform_alm(lmax, mmax, 102))):
        a = a.copy()
        a[: lmax + 1] += 0.25j  # Im a_l0 must be ignored
        say(f"{name} alm2map {kind} lmax={lmax} mmax={mmax} nrings={g.nrings}")
        ref = oracle.alm2map(lmax, mmax, g, a)
        got = host(sht.alm2map(dev(a), g, lmax, mmax))
        if np.linalg.norm(ref) > 0:
            assert relrms(got, ref) <= TOL, (name, kind, relrms(got, ref))
        assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    s = si.random_map(g, 103)
    say(f"{name} map2alm lmax={lmax} mmax={mmax}")
    ref = oracle.map2alm(lmax, mmax, g, s)
    got = host(sht.map2alm(dev(s), g, lmax, mmax))
    assert relrms(got, ref) <= TOL, (name, relrms(got, ref))
    assert np.all(got[: lmax + 1].imag == 0.0)


@pytest.mark.parametrize("case", SMALL_CASES[6:11], ids=[c[0] for c in SMALL_CASES[6:11]])
def test_small_stages(sht, case):
    name, mk, lmax, mmax = case
    g = mk()
    a = si.uniform_alm(lmax, mmax, 7)
    say(f"{name} alm2delta")
    ref = oracle.delta_syn(lmax, mmax, g, a)
    got = host(sht.alm2delta(dev(a), g, lmax, mmax))
    assert relrms(got, ref) <= TOL
    rng = np.random.default_rng(8)
    d = rng.standard_normal((g.nrings, mmax + 1)) + 1j * rng.standard_normal((g.nrings, mmax + 1))
    say(f"{name} delta2map")
    ref = oracle.delta2map(mmax, g, d)
    got = host(sht.delta2map(dev(d), g, mmax))
    assert relrms(got, ref) <= TOL
    s = si.random_map(g, 9)
    say(f"{name} map2delta")
    ref = oracle.map2delta(mmax, g, s)
    got = host(sht.map2delta(dev(s), g, mmax))
    assert relrms(got, ref) <= TOL
    say(f"{name} delta2alm")
    ref = oracle.delta2alm(lmax, mmax, g, d)
    got = host(sht.delta2alm(dev(d), g, lmax, mmax))
    assert relrms(got, ref) <= TOL


def test_config1_gl_lmax256_full(sht):
    lmax = 256
    g = si.gauss_legendre(257, 513)
    a = si.powerlaw_alm(lmax, lmax, si.config_seed(1))
    say("config1 alm2map lmax=256 GL 257x513")
    ref = oracle.alm2map(lmax, lmax, g, a)
    got = host(sht.alm2map(dev(a), g, lmax))
    assert relrms(got, ref) <= TOL, relrms(got, ref)
    say("config1 round trip")
    back = host(sht.map2alm(dev(got), g, lmax))
    assert relrms(back, a) <= 1e-13


def _ring_errors(g, got, ref, rings):
    errs = {}
    for r in rings:
        sl = slice(g.ofs[r], g.ofs[r] + g.nphi[r])
        errs[int(r)] = relrms(got[sl], ref[sl])
    worst = sorted(errs.items(), key=lambda kv: -kv[1])[:5]
    say("worst rings (ring, rel rms): " + ", ".join(f"({r}, {e:.2e})" for r, e in worst))
    return errs


def _ring_pixels(g, rings):
    return np.concatenate([np.arange(g.ofs[r], g.ofs[r] + g.nphi[r]) for r in rings])


def _m_entries(lmax, ms):
    return np.concatenate([si.alm_index(np.arange(m, lmax + 1), m, lmax) for m in ms])


def test_config2_healpix1024_lmax2048_full_map(sht):
    """Whole-map relative RMS against the oracle on every ring (the oracle
    takes ~20 s on 8 host cores; cached for the other config-2 tests)."""
    g, lmax, a = oc.config2()
    say("config2 alm2map full size, full oracle")
    got = host(sht.alm2map(dev(a), g, lmax))
    ref = oc.config2_map()
    err = relrms(got, ref)
    say(f"config2 alm2map whole-map rel rms {err:.3e}")
    assert err <= TOL
    # Per ring: a southern ring paired with its northern mirror is evaluated
    # at the northern ring's cos/sin; its own colatitude, rounded from
    # pi - theta_n, differs by up to half an ulp of pi, which moves the
    # values of the 4-pixel rings next to the south pole by a few 1e-12.
    errs = _ring_errors(g, got, ref, range(g.nrings))
    north = [e for r, e in errs.items() if r < g.nrings // 2 + 1]
    assert max(north) <= TOL
    assert max(errs.values()) <= 1e-11


def test_config2_map2alm_all_m(sht):
    """Analysis at full size against the oracle's map2alm over every m: the
    whole a_lm set at 1e-12 relative RMS, and every m column on its own."""
    g, lmax, _ = oc.config2()
    s, ref_a = oc.config2_analysis_input()
    say("config2 map2alm full size, all m against the oracle")
    got_a = host(sht.map2alm(dev(s), g, lmax))
    err = relrms(got_a, ref_a)
    say(f"config2 map2alm whole-a_lm rel rms {err:.3e}")
    assert err <= TOL
    assert np.all(got_a[: lmax + 1].imag == 0.0)
    worst = 0.0
    for m in range(lmax + 1):
        i0, i1 = si.alm_index(m, m, lmax), si.alm_index(lmax, m, lmax) + 1
        worst = max(worst, relrms(got_a[i0:i1], ref_a[i0:i1]))
    say(f"config2 map2alm worst m column rel rms {worst:.3e}")
    assert worst <= TOL

def test_deterministic_bitwise(sht):
    lmax = 128
    g = si.healpix(64)
    a = si.powerlaw_alm(lmax, lmax, 5)
    s = si.random_map(g, 6)
    say("determinism")
    m1 = host(sht.alm2map(dev(a), g, lmax))
    m2 = host(sht.alm2map(dev(a), g, lmax))
    assert np.array_equal(m1, m2)
    a1 = host(sht.map2alm(dev(s), g, lmax))
    a2 = host(sht.map2alm(dev(s), g, lmax))
    assert np.array_equal(a1, a2)


@pytest.mark.parametrize("nmaps", [2, 3, 9])
def test_multiple_maps_match_single(sht, nmaps):
    """Several maps per call share each recurrence (synthesis: 2, 4 or 8 maps
    per workgroup; 9 maps leave a ragged last group): every map is the same
    bits as its own single-map call, in both directions."""
    import torch
    lmax = 48
    g = si.healpix(16)
    al = np.stack([si.powerlaw_alm(lmax, lmax, 30 + i) for i in range(nmaps)])
    say(f"nmaps={nmaps} alm2map")
    many = host(sht.alm2map(dev(al), g, lmax))
    for i in range(nmaps):
        one = host(sht.alm2map(dev(al[i]), g, lmax))
        assert np.array_equal(many[i], one), i
    say(f"nmaps={nmaps} map2alm")
    back = host(sht.map2alm(torch.from_numpy(many).cuda(), g, lmax))
    for i in range(nmaps):
        one = host(sht.map2alm(dev(many[i]), g, lmax))
        assert np.array_equal(back[i], one), i


def test_workspace_too_small_raises(sht):
    import torch
    g = si.healpix(4)
    a = dev(si.powerlaw_alm(8, 8, 1))
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(sht.ShtError) as e:
        sht.alm2map(a, g, 8, ws=ws)
    assert e.value.code == sht.SHT_EWORKSPACE


def test_plan_cache_eviction_and_shutdown(sht):
    """More geometries than the plan cache holds (LRU eviction of plans and
    their start tables), then sht_shutdown and a fresh start: results stay
    equal to the oracle throughout."""
    lmax = 12
    a = si.uniform_alm(lmax, lmax, 41)
    geoms = [si.gauss_legendre(13, 25 + k) for k in range(36)]  # 36 distinct plans (cache holds 32)
    say("plan cache: 36 geometries")
    for k, g in enumerate(geoms):
        got = host(sht.alm2map(dev(a), g, lmax))
        ref = oracle.alm2map(lmax, lmax, g, a)
        assert relrms(got, ref) <= TOL, k
    say("plan cache: first geometry again after eviction")
    got = host(sht.alm2map(dev(a), geoms[0], lmax))
    assert relrms(got, oracle.alm2map(lmax, lmax, geoms[0], a)) <= TOL
    say("shutdown and re-initialise")
    sht.shutdown()
    got = host(sht.alm2map(dev(a), geoms[1], lmax))
    assert relrms(got, oracle.alm2map(lmax, lmax, geoms[1], a)) <= TOL
    s = si.random_map(geoms[2], 42)
    got = host(sht.map2alm(dev(s), geoms[2], lmax))
    assert relrms(got, oracle.map2alm(lmax, lmax, geoms[2], s)) <= TOL


def test_start_table_serves_smaller_sizes(sht):
    """A start table built for (lmax, mmax) is reused for smaller lmax and mmax
    on the same geometry."""
    g = si.healpix(8)
    for lmax, mmax in ((30, 30), (20, 20), (30, 12), (17, 5)):
        a = si.powerlaw_alm(lmax, mmax, 50 + lmax + mmax)
        say(f"start-table reuse lmax={lmax} mmax={mmax}")
        got = host(sht.alm2map(dev(a), g, lmax, mmax))
        assert relrms(got, oracle.alm2map(lmax, mmax, g, a)) <= TOL
        s = si.random_map(g, 60 + lmax)
        got = host(sht.map2alm(dev(s), g, lmax, mmax))
        assert relrms(got, oracle.map2alm(lmax, mmax, g, s)) <= TOL


def test_concurrent_host_threads_and_streams(sht):
    """Two host threads, each on its own stream and geometry, call the library
    at the same time (plan builds included); each result equals its serial run."""
    import threading
    import torch
    cases = [(si.healpix(16), 40, 71), (si.gauss_legendre(41, 81), 40, 72)]
    serial = []
    for g, lmax, seed in cases:
        a = dev(si.powerlaw_alm(lmax, lmax, seed))
        serial.append(host(sht.alm2map(a, g, lmax)))
    sht.shutdown()  # both threads build their plans concurrently
    out = [None, None]
    errs = []

    def run(i):
        try:
            g, lmax, seed = cases[i]
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                a = dev(si.powerlaw_alm(lmax, lmax, seed))
                for _ in range(3):
                    m = sht.alm2map(a, g, lmax, stream=st)
                st.synchronize()
                out[i] = m.cpu().numpy()
        except Exception as e:  # reported below
            errs.append(e)

    say("two host threads")
    ts = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert not errs, errs
    for i in range(2):
        assert np.array_equal(out[i], serial[i]), i


def test_stage_entry_points_several_maps(sht):
    lmax = 20
    g = si.healpix(8)
    al = np.stack([si.uniform_alm(lmax, lmax, 80 + i) for i in range(2)])
    say("alm2delta / delta2alm with nmaps=2")
    d = host(sht.alm2delta(dev(al), g, lmax))
    for i in range(2):
        assert relrms(d[i], oracle.delta_syn(lmax, lmax, g, al[i])) <= TOL
    back = host(sht.delta2alm(dev(d), g, lmax))
    for i in range(2):
        assert relrms(back[i], oracle.delta2alm(lmax, lmax, g, d[i])) <= TOL
    say("delta2map / map2delta with nmaps=2")
    mp = host(sht.delta2map(dev(d), g, lmax))
    for i in range(2):
        assert relrms(mp[i], oracle.delta2map(lmax, g, d[i])) <= TOL
    dd = host(sht.map2delta(dev(mp), g, lmax))
    for i in range(2):
        assert relrms(dd[i], oracle.map2delta(lmax, g, mp[i])) <= TOL


def test_ring_stages_prime_radix_lengths(sht):
    """Ring lengths whose prime factors above 5 run the mirror-paired direct
    stage, in every length class: 4095 = 3^2 5 7 13 and 8190 = 2 3^2 5 7 13
    (radix 13 fills the most work items per thread, in the 4096 and 8192
    classes), 8173 = 11 x 743 (a 743-point stage: Bluestein would exceed the
    largest class), 1001 = 7 11 13, 4 x 61, 4 x 97, and for contrast 4091
    (prime: Bluestein on 8192 points) and 139 (prime).  Both ring stages
    against the oracle's plain DFTs, rings at arbitrary colatitudes (no
    mirror pairs) and phases."""
    nphi = np.array([4095, 8190, 8173, 1001, 244, 388, 4091, 139], dtype=np.int32)
    nr = nphi.size
    rng = np.random.default_rng(41)
    th = np.sort(rng.uniform(0.05, math.pi - 0.05, nr))
    g = si._pack(th, nphi, rng.uniform(-1.0, 2.0, nr), rng.uniform(0.2, 1.0, nr), "prime_lengths")
    for mmax in (40, 600):
        d = rng.standard_normal((nr, mmax + 1)) + 1j * rng.standard_normal((nr, mmax + 1))
        say(f"prime ring lengths delta2map mmax={mmax}")
        ref = oracle.delta2map(mmax, g, d)
        got = host(sht.delta2map(dev(d), g, mmax))
        for r in range(nr):
            o, n = int(g.ofs[r]), int(nphi[r])
            assert relrms(got[o:o + n], ref[o:o + n]) <= TOL, (mmax, n, relrms(got[o:o + n], ref[o:o + n]))
        s_map = si.random_map(g, 42 + mmax)
        say(f"prime ring lengths map2delta mmax={mmax}")
        ref = oracle.map2delta(mmax, g, s_map)
        got = host(sht.map2delta(dev(s_map), g, mmax))
        for r in range(nr):
            assert relrms(got[r], ref[r]) <= TOL, (mmax, int(nphi[r]), relrms(got[r], ref[r]))


def test_ring_stages_bluestein_shortest_length(sht):
    """Bluestein at its shortest cyclic length L = 2n - 2 (5-smooth n - 1):
    641 -> 1280, 1153 -> 2304, 2049 = 3 x 683 -> 4096 and 3457 -> 6912, one
    per length class from 2048 up; offsets +-(n-1) of the even chirp share
    one index there.  For contrast 4091 (L = 8192 > 2n - 2) and 1021 (L =
    2048).  Both ring stages against the oracle's plain DFTs, rings at
    arbitrary colatitudes and phases, with mmax below and above n / 2 (bins
    folding several m)."""
    nphi = np.array([641, 1153, 2049, 3457, 4091, 1021], dtype=np.int32)
    nr = nphi.size
    rng = np.random.default_rng(43)
    th = np.sort(rng.uniform(0.05, math.pi - 0.05, nr))
    g = si._pack(th, nphi, rng.uniform(-1.0, 2.0, nr), rng.uniform(0.2, 1.0, nr), "bluestein_short")
    for mmax in (300, 2500):
        d = rng.standard_normal((nr, mmax + 1)) + 1j * rng.standard_normal((nr, mmax + 1))
        say(f"Bluestein L = 2n - 2 delta2map mmax={mmax}")
        ref = oracle.delta2map(mmax, g, d)
        got = host(sht.delta2map(dev(d), g, mmax))
        for r in range(nr):
            o, n = int(g.ofs[r]), int(nphi[r])
            assert relrms(got[o:o + n], ref[o:o + n]) <= TOL, (mmax, n, relrms(got[o:o + n], ref[o:o + n]))
        s_map = si.random_map(g, 44 + mmax)
        say(f"Bluestein L = 2n - 2 map2delta mmax={mmax}")
        ref = oracle.map2delta(mmax, g, s_map)
        got = host(sht.map2delta(dev(s_map), g, mmax))
        for r in range(nr):
            assert relrms(got[r], ref[r]) <= TOL, (mmax, int(nphi[r]), relrms(got[r], ref[r]))


def test_gl_lmax2048_direct_prime_radices(sht):
    """Gauss-Legendre, 2049 rings of 4097 = 17 x 241 points, lmax = 2048: the
    ring transforms run as direct radix-17 and radix-241 stages (by the plan's
    cost model cheaper than Bluestein on 8192 points, the largest class).  FP64 against the oracle on
    every fourth ring (synthesis) and every fourth m (analysis of a white-noise
    map), each set aggregated at 1e-12, and per ring / per m column."""
    lmax = 2048
    g = si.gauss_legendre(lmax + 1, 2 * lmax + 1)
    a = si.powerlaw_alm(lmax, lmax, si.config_seed(4))
    say("GL 2049x4097 lmax 2048 alm2map / map2alm")
    m_h = host(sht.alm2map(dev(a), g, lmax))
    rings = np.arange(0, g.nrings, 4)
    rings = np.union1d(rings, [1, g.nrings - 2, g.nrings - 1]).astype(np.int32)
    ref = oracle.alm2map(lmax, lmax, g, a, rings=rings)
    px = _ring_pixels(g, rings)
    err = relrms(m_h[px], ref[px])
    say(f"GL2049 alm2map rel rms over {len(rings)} rings {err:.3e}")
    assert err <= TOL
    # per ring: 3e-12 in the north (a 4097-pixel ring next to the pole sums
    # 2049 recurrence terms of rounding on its own); southern rings are
    # evaluated at the mirrored northern colatitude (half an ulp of pi away)
    errs = _ring_errors(g, m_h, ref, rings)
    for r, e in errs.items():
        assert e <= (3e-12 if r < g.nrings // 2 else 2e-11), (r, e)
    # analysis of a seeded white-noise map on the same grid
    ms = np.union1d(np.arange(0, lmax + 1, 4), [1, lmax - 1, lmax]).astype(np.int32)
    src = si.random_map(g, 4049)
    back = host(sht.map2alm(dev(src), g, lmax))
    ref_a = oracle.map2alm(lmax, lmax, g, src, ms=ms)
    ix = _m_entries(lmax, ms)
    err = relrms(back[ix], ref_a[ix])
    say(f"GL2049 map2alm rel rms over {len(ms)} m {err:.3e}")
    assert err <= TOL
    for m in ms:
        idx = si.alm_index(np.arange(m, lmax + 1), m, lmax)
        assert relrms(back[idx], ref_a[idx]) <= 3e-12, (int(m), relrms(back[idx], ref_a[idx]))
    # Gauss-Legendre quadrature is exact at this band limit: analysis of the
    # synthesised map returns the input
    back = host(sht.map2alm(dev(m_h), g, lmax))
    assert relrms(back, a) <= 1e-11, relrms(back, a)


@pytest.mark.parametrize("nmaps", [1, 3])
def test_fp64_three_slots_per_lane_gl1025(sht, nmaps):
    """Gauss-Legendre 1025 x 2049 at lmax 1024: 513 ring slots, which the FP64
    kernels hold at 3 per lane (synthesis of one map, two-map synthesis with
    a ragged last pair of maps, analysis).  Every map against the oracle on
    every eighth ring and every eighth m at 1e-12, and the exact Gauss-Legendre
    round trip."""
    lmax = 1024
    g = si.gauss_legendre(lmax + 1, 2 * lmax + 1)
    a = np.stack([si.powerlaw_alm(lmax, lmax, si.config_seed(3, 40 + i)) for i in range(nmaps)])
    say(f"GL1025x2049 lmax 1024 FP64, {nmaps} map(s)")
    m_h = host(sht.alm2map(dev(a), g, lmax)).reshape(nmaps, -1)
    rings = np.union1d(np.arange(0, g.nrings, 8), [1, g.nrings // 2, g.nrings - 1]).astype(np.int32)
    px = _ring_pixels(g, rings)
    for i in range(nmaps):
        ref = oracle.alm2map(lmax, lmax, g, a[i], rings=rings)
        err = relrms(m_h[i][px], ref[px])
        say(f"map {i}: alm2map rel rms over {len(rings)} rings {err:.3e}")
        assert err <= TOL, (i, err)
    src = np.stack([si.random_map(g, 5000 + i) for i in range(nmaps)])
    back = host(sht.map2alm(dev(src), g, lmax)).reshape(nmaps, -1)
    ms = np.union1d(np.arange(0, lmax + 1, 8), [1, lmax]).astype(np.int32)
    ix = _m_entries(lmax, ms)
    for i in range(nmaps):
        ref_a = oracle.map2alm(lmax, lmax, g, src[i], ms=ms)
        err = relrms(back[i][ix], ref_a[ix])
        say(f"map {i}: map2alm rel rms over {len(ms)} m {err:.3e}")
        assert err <= TOL, (i, err)
    rt = host(sht.map2alm(dev(m_h), g, lmax)).reshape(nmaps, -1)
    for i in range(nmaps):
        assert relrms(rt[i], a[i]) <= 1e-11, (i, relrms(rt[i], a[i]))


def test_near_mirror_ring_pair_is_not_paired(sht):
    """A ring pair 5e-15 rad (about 11 ulp of pi) off mirror is two slots,
    each evaluated at its own colatitude, so every ring matches the oracle at
    1e-12.  The a_lm have m = 0 zeroed, so the near-polar rings are dominated
    by m = 1, whose value scales with sin(theta): had the pair been joined,
    the southern ring (theta_n = 1e-3) would be evaluated at the northern
    ring's sin(theta), 5e-15 / 1e-3 relative off, which the oracle puts at
    4.9e-12 on that ring."""
    pi_l = np.longdouble("3.14159265358979323846264338327950288")
    lmax = 64
    g0 = si.gauss_legendre(20, 129)
    th = g0.theta.copy()
    th[0] = 1e-3
    th[-1] = float(pi_l - np.longdouble(1e-3)) + 5e-15
    assert abs(float(np.longdouble(th[0]) + np.longdouble(th[-1]) - pi_l)) > 4e-15
    th[1] = 0.3
    th[-2] = float(pi_l - np.longdouble(0.3))  # an exact (rounded) mirror: still one slot
    g = si._pack(th, g0.nphi, np.linspace(0.0, 0.3, g0.nrings), g0.weight, "near_mirror")
    a = si.uniform_alm(lmax, lmax, 17)
    a[: lmax + 1] = 0.0
    say("near-mirror ring pair: alm2map and map2alm against the oracle")
    got = host(sht.alm2map(dev(a), g, lmax))
    ref = oracle.alm2map(lmax, lmax, g, a)
    errs = _ring_errors(g, got, ref, range(g.nrings))
    assert max(errs.values()) <= TOL, errs
    s = si.random_map(g, 18)
    got_a = host(sht.map2alm(dev(s), g, lmax))
    assert relrms(got_a, oracle.map2alm(lmax, lmax, g, s)) <= TOL
