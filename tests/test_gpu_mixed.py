"""GPU parity of the mixed-precision transforms (SHT_MIXED) against the oracle.

The recurrence stays FP64 and only lambda_lm, the c-scaled a_lm (synthesis)
or the pair sums of Delta (analysis), and the matrix-core sums are FP32, so
the bar is the batched-mixed target: relative RMS <= 1e-6 of every map (or
a_lm set) against the FP64 oracle and against the FP64 HIP path, itself
pinned to 1e-12.  Synthesis batches of 12, 17 and 40 maps take the column
widths of its kernel (16 and 32 maps per wave) and a partly filled last
column group; analysis groups 8 maps and 2048 ring pairs per workgroup.
Below 8 maps SHT_MIXED runs the FP64 kernels (the same bits as flags 0); the
stage calls with map-minor Delta take the mixed kernels at any batch size,
which covers 1 and 3 maps and 8 maps per wave.
"""
import sys

import numpy as np
import pytest

import oracle
import sht_inputs as si

import _oracle_cache as oc

pytestmark = pytest.mark.gpu

MX_TOL = 1e-6


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


def batch(lmax, mmax, nmaps, seed):
    """Power-law and uniform a_lm in turn, Im a_l0 set (it must be ignored)."""
    out = np.empty((nmaps, si.nalm(lmax, mmax)), dtype=np.complex128)
    for i in range(nmaps):
        a = si.powerlaw_alm(lmax, mmax, seed + i) if i % 2 == 0 else si.uniform_alm(lmax, mmax, seed + i)
        a[: lmax + 1] += 0.25j
        out[i] = a
    return out


MX_CASES = [
    # (name, geometry builder, lmax, mmax, nmaps)
    ("gl0_1", lambda: si.gauss_legendre(1, 1), 0, 0, 1),
    ("gl7_mless_3", lambda: si.gauss_legendre(8, 9), 7, 4, 3),
    ("gl31_12", lambda: si.gauss_legendre(32, 63), 31, 31, 12),
    ("gl64_odd_3", lambda: si.gauss_legendre(65, 129), 64, 64, 3),
    ("hp8_alias_12", lambda: si.healpix(8), 40, 40, 12),
    ("hp16_40", lambda: si.healpix(16), 32, 32, 40),
    ("hp32_ragged_17", lambda: si.healpix(32), 77, 61, 17),
    ("random_poles_9", lambda: si._pack(np.array([0.0, 0.4, 1.2, np.pi / 2, 2.0, np.pi]),
                                        np.array([1, 5, 16, 3, 9, 2], dtype=np.int32),
                                        np.array([0.0, 0.1, 2.0, -1.0, 0.5, 0.0]),
                                        np.ones(6), "poles"), 12, 12, 9),
    ("gl_bluestein_40", lambda: si.gauss_legendre(70, 139), 69, 69, 40),
    # 300 unpaired rings: two 256-pair tiles, the second ragged
    ("random300_8", lambda: si._pack(np.sort(np.random.default_rng(3).uniform(0, np.pi, 300)),
                                     np.full(300, 9, dtype=np.int32), np.zeros(300), np.ones(300), "r300"),
     20, 20, 8),
]


@pytest.mark.parametrize("case", MX_CASES, ids=[c[0] for c in MX_CASES])
def test_mixed_alm2map_small(sht, case):
    name, mk, lmax, mmax, nmaps = case
    g = mk()
    a = batch(lmax, mmax, nmaps, 500)
    say(f"mixed alm2map {name} lmax={lmax} mmax={mmax} nrings={g.nrings} nmaps={nmaps}")
    got = host(sht.alm2map(dev(a), g, lmax, mmax, flags=sht.SHT_MIXED))
    f64 = host(sht.alm2map(dev(a), g, lmax, mmax))
    for i in range(nmaps):
        ref = oracle.alm2map(lmax, mmax, g, a[i])
        if np.linalg.norm(ref) == 0:
            assert np.all(got[i] == 0.0)
            continue
        assert relrms(got[i], ref) <= MX_TOL, (name, i, relrms(got[i], ref))
        assert relrms(got[i], f64[i]) <= MX_TOL, (name, i, relrms(got[i], f64[i]))


def test_mixed_below_8_maps_runs_the_fp64_kernels(sht):
    """With fewer than 8 maps the matrix-core columns would mostly idle and
    FP32 vector arithmetic is no faster than FP64, so SHT_MIXED runs the FP64
    kernels: the same bits as flags 0 in both directions."""
    lmax, g = 40, si.healpix(8)
    for nmaps in (1, 3, 7):
        say(f"mixed below 8 maps: nmaps={nmaps}")
        a = dev(batch(lmax, lmax, nmaps, 800 + nmaps))
        assert np.array_equal(host(sht.alm2map(a, g, lmax, flags=sht.SHT_MIXED)), host(sht.alm2map(a, g, lmax)))
        mp = dev(np.stack([si.random_map(g, 820 + i) for i in range(nmaps)]))
        assert np.array_equal(host(sht.map2alm(mp, g, lmax, flags=sht.SHT_MIXED)), host(sht.map2alm(mp, g, lmax)))


@pytest.mark.parametrize("case", [MX_CASES[0], MX_CASES[1], MX_CASES[3], MX_CASES[9]],
                         ids=[MX_CASES[0][0], MX_CASES[1][0], MX_CASES[3][0], MX_CASES[9][0]])
def test_mixed_kernels_small_batches_map_minor(sht, case):
    """Map-minor Delta takes the mixed kernels at any batch size: 1, 3 and 8
    maps (lmax 0, mmax < lmax, odd ring count, ragged pair tile) through the
    Legendre stage calls, against the oracle's Delta and a_lm."""
    name, mk, lmax, mmax, nmaps = case
    g = mk()
    a = batch(lmax, mmax, nmaps, 900)
    X = sht.SHT_MIXED | sht.SHT_DELTA_MAP_MINOR
    say(f"mixed kernels, map-minor stage calls: {name} nmaps={nmaps}")
    d = host(sht.alm2delta(dev(a), g, lmax, mmax, flags=X))  # [nrings][mmax+1][nmaps]
    refs = [oracle.delta_syn(lmax, mmax, g, a[i]) for i in range(nmaps)]
    for i in range(nmaps):
        if np.linalg.norm(refs[i]) > 0:
            assert relrms(d[:, :, i], refs[i]) <= MX_TOL, (name, i, relrms(d[:, :, i], refs[i]))
    dd = np.ascontiguousarray(np.stack(refs, axis=-1))
    back = host(sht.delta2alm(dev(dd), g, lmax, mmax, flags=X))
    for i in range(nmaps):
        ref = oracle.delta2alm(lmax, mmax, g, refs[i])
        if np.linalg.norm(ref) > 0:
            assert relrms(back[i], ref) <= MX_TOL, (name, i, relrms(back[i], ref))


@pytest.mark.parametrize("case", [MX_CASES[4], MX_CASES[6]], ids=[MX_CASES[4][0], MX_CASES[6][0]])
def test_mixed_alm2delta(sht, case):
    name, mk, lmax, mmax, nmaps = case
    g = mk()
    a = batch(lmax, mmax, nmaps, 600)
    say(f"mixed alm2delta {name} nmaps={nmaps}")
    got = host(sht.alm2delta(dev(a), g, lmax, mmax, flags=sht.SHT_MIXED))
    for i in range(nmaps):
        ref = oracle.delta_syn(lmax, mmax, g, a[i])
        assert relrms(got[i], ref) <= MX_TOL, (name, i, relrms(got[i], ref))


def test_mixed_is_deterministic_and_batch_independent(sht):
    """The same map gives the same bits alone in its column group and inside
    a larger batch (columns of the matrix products are independent, and the
    ring stages pair the same two adjacent maps), and on a repeated call."""
    lmax, g = 40, si.healpix(8)
    a = batch(lmax, lmax, 40, 700)
    say("mixed determinism hp8 lmax=40 nmaps=40")
    full = host(sht.alm2map(dev(a), g, lmax, flags=sht.SHT_MIXED))
    again = host(sht.alm2map(dev(a), g, lmax, flags=sht.SHT_MIXED))
    assert np.array_equal(full, again)
    # maps 32..39 form the second group of 32; alone they are a batch of 8
    part = host(sht.alm2map(dev(a[32:]), g, lmax, flags=sht.SHT_MIXED))
    assert np.array_equal(part, full[32:])
    maps = dev(np.stack([si.random_map(g, 710 + i) for i in range(40)]))
    fa = host(sht.map2alm(maps, g, lmax, flags=sht.SHT_MIXED))
    pa = host(sht.map2alm(maps[32:].contiguous(), g, lmax, flags=sht.SHT_MIXED))
    assert np.array_equal(pa, fa[32:])


ANA_CASES = [
    # (name, geometry builder, lmax, mmax, nmaps)
    ("gl0_1", lambda: si.gauss_legendre(1, 1), 0, 0, 1),
    ("gl7_mless_3", lambda: si.gauss_legendre(8, 9), 7, 4, 3),
    ("gl64_odd_9", lambda: si.gauss_legendre(65, 129), 64, 64, 9),
    ("hp8_alias_8", lambda: si.healpix(8), 40, 40, 8),
    ("hp32_ragged_17", lambda: si.healpix(32), 77, 61, 17),
    ("random_poles_5", MX_CASES[7][1], 12, 12, 5),
    ("gl_bluestein_12", lambda: si.gauss_legendre(70, 139), 69, 69, 12),
    # 2300 unpaired rings: two groups of 2048 pairs, partial sums combined
    ("random2300_3", lambda: si._pack(np.sort(np.random.default_rng(11).uniform(0, np.pi, 2300)),
                                      np.full(2300, 7, dtype=np.int32), np.zeros(2300),
                                      np.random.default_rng(12).uniform(0.1, 1.0, 2300), "r2300"), 24, 24, 3),
]


@pytest.mark.parametrize("case", ANA_CASES, ids=[c[0] for c in ANA_CASES])
def test_mixed_map2alm_small(sht, case):
    name, mk, lmax, mmax, nmaps = case
    g = mk()
    maps = np.stack([si.random_map(g, 800 + i) for i in range(nmaps)])
    say(f"mixed map2alm {name} lmax={lmax} mmax={mmax} nrings={g.nrings} nmaps={nmaps}")
    got = host(sht.map2alm(dev(maps), g, lmax, mmax, flags=sht.SHT_MIXED))
    f64 = host(sht.map2alm(dev(maps), g, lmax, mmax))
    for i in range(nmaps):
        ref = oracle.map2alm(lmax, mmax, g, maps[i])
        assert relrms(got[i], ref) <= MX_TOL, (name, i, relrms(got[i], ref))
        assert relrms(got[i], f64[i]) <= MX_TOL, (name, i, relrms(got[i], f64[i]))
        assert np.all(got[i][: lmax + 1].imag == 0.0)


def test_mixed_delta2alm(sht):
    lmax, mmax, g, nmaps = 77, 61, si.healpix(32), 10
    rng = np.random.default_rng(900)
    d = rng.standard_normal((nmaps, g.nrings, mmax + 1)) + 1j * rng.standard_normal((nmaps, g.nrings, mmax + 1))
    say(f"mixed delta2alm hp32 lmax={lmax} mmax={mmax} nmaps={nmaps}")
    got = host(sht.delta2alm(dev(d), g, lmax, mmax, flags=sht.SHT_MIXED))
    for i in range(nmaps):
        ref = oracle.delta2alm(lmax, mmax, g, d[i])
        assert relrms(got[i], ref) <= MX_TOL, (i, relrms(got[i], ref))


def test_mixed_round_trip_gl(sht):
    """On a Gauss-Legendre grid analysis inverts synthesis for band-limited
    a_lm (exact quadrature): mixed there and back stays within the bar."""
    lmax, nmaps = 63, 12
    g = si.gauss_legendre(lmax + 1, 2 * lmax + 1)
    a = batch(lmax, lmax, nmaps, 950)
    a[:, : lmax + 1] = a[:, : lmax + 1].real
    say("mixed round trip GL lmax=63 nmaps=12")
    mp = sht.alm2map(dev(a), g, lmax, flags=sht.SHT_MIXED)
    back = host(sht.map2alm(mp, g, lmax, flags=sht.SHT_MIXED))
    for i in range(nmaps):
        assert relrms(back[i], a[i]) <= 2 * MX_TOL, (i, relrms(back[i], a[i]))


def test_mixed_full_size_healpix1024_lmax2048_64maps(sht):
    """The batched configuration of the benchmark: 64 power-law maps on
    HEALPix N_side = 1024, lmax = 2048.  Map 0 against the oracle over every
    pixel, and three maps against the FP64 HIP path over every pixel; in
    analysis, map 0 (the oracle's config-2 analysis input) against the oracle
    over every a_lm, and three maps against the FP64 HIP path."""
    import torch
    lmax, nmaps = 2048, 64
    g = si.healpix(1024)
    say("mixed alm2map full size: healpix 1024 lmax 2048 nmaps 64")
    alm = torch.empty((nmaps, si.nalm(lmax, lmax)), dtype=torch.complex128, device="cuda")
    for i in range(nmaps):
        alm[i] = dev(si.powerlaw_alm(lmax, lmax, si.config_seed(2, i)))
    got = sht.alm2map(alm, g, lmax, flags=sht.SHT_MIXED)
    g0 = host(got[0])
    err0 = relrms(g0, oc.config2_map())
    say(f"mixed alm2map map 0 vs oracle, whole map: {err0:.3e}")
    assert err0 <= MX_TOL
    for i in (0, 37, 63):
        ref = host(sht.alm2map(alm[i].contiguous(), g, lmax))
        gi = host(got[i])
        assert relrms(gi, ref) <= MX_TOL, (i, relrms(gi, ref))
    say("mixed map2alm full size: healpix 1024 lmax 2048 nmaps 64")
    maps = sht.alm2map(alm, g, lmax)
    s0, ref_a0 = oc.config2_analysis_input()
    maps[0] = dev(s0)
    back = sht.map2alm(maps, g, lmax, flags=sht.SHT_MIXED)
    b0 = host(back[0])
    err0 = relrms(b0, ref_a0)
    say(f"mixed map2alm map 0 vs oracle, all a_lm: {err0:.3e}")
    assert err0 <= MX_TOL
    for i in (0, 37, 63):
        ref = host(sht.map2alm(maps[i].contiguous(), g, lmax))
        bi = host(back[i])
        assert relrms(bi, ref) <= MX_TOL, (i, relrms(bi, ref))


def test_mixed_fp64_block_sums_healpix1024_lmax2048(sht):
    """SHT_MIXED_FP64_SUMS: each 32-l block summed on the matrix cores in a
    fresh FP32 accumulator, the block sums added in FP64 (the compensated
    form of the synthesis l-sum).  8 power-law maps on HEALPix N_side = 1024
    at lmax 2048: map 0 against the oracle over every pixel and every map
    against the FP64 HIP path at 3e-7, below the plain FP32 chain's error."""
    import torch
    lmax, nmaps = 2048, 8
    g = si.healpix(1024)
    say("mixed alm2map with FP64 block sums: healpix 1024 lmax 2048 nmaps 8")
    alm = torch.empty((nmaps, si.nalm(lmax, lmax)), dtype=torch.complex128, device="cuda")
    for i in range(nmaps):
        alm[i] = dev(si.powerlaw_alm(lmax, lmax, si.config_seed(2, i)))
    comp = sht.alm2map(alm, g, lmax, flags=sht.SHT_MIXED | sht.SHT_MIXED_FP64_SUMS)
    plain = sht.alm2map(alm, g, lmax, flags=sht.SHT_MIXED)
    f64 = sht.alm2map(alm, g, lmax)
    err0 = relrms(host(comp[0]), oc.config2_map())
    e_comp = ((comp - f64).norm(dim=1) / f64.norm(dim=1)).cpu().numpy()
    e_plain = ((plain - f64).norm(dim=1) / f64.norm(dim=1)).cpu().numpy()
    say(f"FP64 block sums: map 0 vs oracle {err0:.3e}; vs FP64 max {e_comp.max():.3e} "
        f"(one FP32 chain: max {e_plain.max():.3e})")
    assert err0 <= 3e-7
    assert np.all(e_comp <= 3e-7), e_comp
    assert e_comp.max() < e_plain.max()


SPLIT_CASES = [c for c in MX_CASES if c[4] >= 8]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=[c[0] for c in SPLIT_CASES])
def test_split_bf16_alm2map_small(sht, case):
    """SHT_MIXED_SPLIT_BF16: every map against the oracle and the FP64 HIP
    path at the mixed bar, and no worse than the FP32 matrix-core path on the
    same FP32 operands (1.5x its error + 5e-8): a part of the three-way split
    lost or misplaced would leave about 2^-16 = 1.5e-5 relative.  Also with
    FP64 block sums (8 maps per wave)."""
    name, mk, lmax, mmax, nmaps = case
    g = mk()
    a = batch(lmax, mmax, nmaps, 700)
    sp = sht.SHT_MIXED | sht.SHT_MIXED_SPLIT_BF16
    say(f"split-bf16 alm2map {name} lmax={lmax} mmax={mmax} nrings={g.nrings} nmaps={nmaps}")
    got = host(sht.alm2map(dev(a), g, lmax, mmax, flags=sp))
    got_f64s = host(sht.alm2map(dev(a), g, lmax, mmax, flags=sp | sht.SHT_MIXED_FP64_SUMS))
    f32 = host(sht.alm2map(dev(a), g, lmax, mmax, flags=sht.SHT_MIXED))
    f64 = host(sht.alm2map(dev(a), g, lmax, mmax))
    for i in range(nmaps):
        ref = oracle.alm2map(lmax, mmax, g, a[i])
        if np.linalg.norm(ref) == 0:
            assert np.all(got[i] == 0.0) and np.all(got_f64s[i] == 0.0)
            continue
        for v in (got[i], got_f64s[i]):
            assert relrms(v, ref) <= MX_TOL, (name, i, relrms(v, ref))
            assert relrms(v, f64[i]) <= MX_TOL, (name, i, relrms(v, f64[i]))
        e_sp, e_f32 = relrms(got[i], f64[i]), relrms(f32[i], f64[i])
        assert e_sp <= 1.5 * e_f32 + 5e-8, (name, i, e_sp, e_f32)


def test_split_bf16_alm2delta_map_minor(sht):
    """The split variant through the synthesis stage call with map-minor
    Delta: every map's Delta against the oracle's delta_syn (12 maps, one
    16-map column group with 4 empty columns)."""
    name, mk, lmax, mmax, nmaps = MX_CASES[1]
    g = mk()
    a = batch(lmax, mmax, nmaps, 710)
    say(f"split-bf16 alm2delta map-minor {name} nmaps={nmaps}")
    got = host(sht.alm2delta(dev(a), g, lmax, mmax,
                             flags=sht.SHT_MIXED | sht.SHT_MIXED_SPLIT_BF16 | sht.SHT_DELTA_MAP_MINOR))
    for i in range(nmaps):
        ref = oracle.delta_syn(lmax, mmax, g, a[i])
        assert relrms(got[..., i], ref) <= MX_TOL, (name, i, relrms(got[..., i], ref))


def test_split_bf16_healpix1024_lmax2048(sht):
    """The split variant at full size: 24 power-law maps on HEALPix N_side =
    1024 at lmax 2048 (one 32-map column group per wave, 8 columns empty),
    map 0 against the oracle over every pixel and every map against the FP64
    HIP path at the mixed bar; the analysis calls reject the flag."""
    import torch
    lmax, nmaps = 2048, 24
    g = si.healpix(1024)
    say("split-bf16 alm2map: healpix 1024 lmax 2048 nmaps 24")
    alm = torch.empty((nmaps, si.nalm(lmax, lmax)), dtype=torch.complex128, device="cuda")
    for i in range(nmaps):
        alm[i] = dev(si.powerlaw_alm(lmax, lmax, si.config_seed(2, i)))
    sp = sht.SHT_MIXED | sht.SHT_MIXED_SPLIT_BF16
    got = sht.alm2map(alm, g, lmax, flags=sp)
    f64 = sht.alm2map(alm, g, lmax)
    err0 = relrms(host(got[0]), oc.config2_map())
    e = ((got - f64).norm(dim=1) / f64.norm(dim=1)).cpu().numpy()
    say(f"split-bf16: map 0 vs oracle {err0:.3e}; vs FP64 max {e.max():.3e}")
    assert err0 <= MX_TOL
    assert np.all(e <= MX_TOL), e
    with pytest.raises(sht.ShtError):
        sht.map2alm(got, g, lmax, flags=sp)


def test_mixed_batched_gl1025_lmax1024_64maps(sht):
    """The batched configuration on a Gauss-Legendre grid: 64 power-law maps,
    1025 rings of 2049 points (2049 = 3 x 683: Bluestein), lmax = 1024.  All
    maps against the FP64 HIP path, four maps against the oracle, in both
    directions."""
    import torch
    lmax, nmaps = 1024, 64
    g = si.gauss_legendre(lmax + 1, 2 * lmax + 1)
    say("mixed config GL 1025x2049 lmax 1024 nmaps 64")
    alm = torch.empty((nmaps, si.nalm(lmax, lmax)), dtype=torch.complex128, device="cuda")
    for i in range(nmaps):
        alm[i] = dev(si.powerlaw_alm(lmax, lmax, si.config_seed(3, i)))
    got = sht.alm2map(alm, g, lmax, flags=sht.SHT_MIXED)
    f64 = sht.alm2map(alm, g, lmax)
    err = ((got - f64).norm(dim=1) / f64.norm(dim=1)).cpu().numpy()
    assert np.all(err <= MX_TOL), err.max()
    back = sht.map2alm(f64, g, lmax, flags=sht.SHT_MIXED)
    back64 = sht.map2alm(f64, g, lmax)
    err = ((back - back64).norm(dim=1) / back64.norm(dim=1)).cpu().numpy()
    assert np.all(err <= MX_TOL), err.max()
    for i in (0, 21, 42, 63):
        a = host(alm[i])
        ref = oracle.alm2map(lmax, lmax, g, a)
        assert relrms(host(got[i]), ref) <= MX_TOL, (i, relrms(host(got[i]), ref))
        # Gauss-Legendre quadrature is exact for this band limit: analysis of
        # the FP64 map returns the input a_lm (Im a_l0 = 0 by construction)
        assert relrms(host(back[i]), a) <= MX_TOL, (i, relrms(host(back[i]), a))


@pytest.mark.parametrize("nmaps", [1, 12, 40])
def test_map_minor_delta_layout_is_bitwise_equal(sht, nmaps):
    """SHT_DELTA_MAP_MINOR moves Delta.  From 8 maps on the mixed Legendre
    stages give the same bits in either layout; below 8 maps ring-major
    Delta runs the FP64 kernels (the same bits as flags 0) and map-minor the
    mixed ones (within the mixed tolerance).  The FFT stages pair two
    adjacent maps of one ring in a complex transform instead of the two rings
    of a mirror pair, so they agree to rounding (the ring-major FFT stages are
    pinned to the oracle at 1e-12).  The combined mixed transforms equal the
    stage composition."""
    import torch
    lmax, mmax, g = 77, 61, si.healpix(32)
    MM = sht.SHT_DELTA_MAP_MINOR
    X = sht.SHT_MIXED
    rng = np.random.default_rng(1000 + nmaps)
    say(f"map-minor layout hp32 lmax={lmax} mmax={mmax} nmaps={nmaps}")
    d = dev(rng.standard_normal((nmaps, g.nrings, mmax + 1)) + 1j * rng.standard_normal((nmaps, g.nrings, mmax + 1)))
    d_mm = d.permute(1, 2, 0).contiguous()
    rel = lambda x, y: ((x - y).norm() / y.norm()).item()
    assert rel(sht.delta2map(d_mm, g, mmax, flags=MM), sht.delta2map(d, g, mmax)) <= 1e-14
    mp = dev(np.stack([si.random_map(g, 1100 + i) for i in range(nmaps)]))
    ds = sht.map2delta(mp, g, mmax)
    ds_mm = sht.map2delta(mp, g, mmax, flags=MM)
    assert rel(ds_mm, ds.permute(1, 2, 0)) <= 1e-14
    ds_mm = ds.permute(1, 2, 0).contiguous()  # the same Delta^S in both layouts below
    a = dev(batch(lmax, mmax, nmaps, 1200))
    dx = sht.alm2delta(a, g, lmax, mmax, flags=X)
    dx_mm = sht.alm2delta(a, g, lmax, mmax, flags=X | MM)
    ax = sht.delta2alm(ds, g, lmax, mmax, flags=X)
    ax_mm = sht.delta2alm(ds_mm, g, lmax, mmax, flags=X | MM)
    if nmaps >= 8:
        assert torch.equal(dx.permute(1, 2, 0), dx_mm)
        assert torch.equal(ax, ax_mm)
    else:
        assert torch.equal(dx, sht.alm2delta(a, g, lmax, mmax))
        assert torch.equal(ax, sht.delta2alm(ds, g, lmax, mmax))
        assert rel(dx_mm, dx.permute(1, 2, 0)) <= MX_TOL
        assert rel(ax_mm, ax) <= MX_TOL
    # the combined mixed calls equal the stage composition: synthesis keeps
    # its Delta map-minor from 8 maps on (whole 128-byte lines), ring-major
    # below; analysis ring-major
    syn_stages = (sht.delta2map(dx_mm, g, mmax, flags=MM) if nmaps >= 8 else sht.delta2map(dx, g, mmax))
    assert torch.equal(sht.alm2map(a, g, lmax, mmax, flags=X), syn_stages)
    assert torch.equal(sht.map2alm(mp, g, lmax, mmax, flags=X), ax)


def test_healpix2048_lmax4096_fp64_and_mixed(sht):
    """lmax = 4096 on HEALPix N_side = 2048 (8191 rings, 4096 ring pairs: two
    analysis groups and the combine kernel at full size).  FP64 against the
    oracle on every eighth ring (synthesis) and every eighth m (analysis of a
    white-noise map), each set aggregated at 1e-12; a mixed batch of 8 maps
    against the FP64 path in both directions: synthesis at 5e-7 (its 32-l
    block sums are added in FP64 above lmax 2048), analysis at 1e-6."""
    import torch
    lmax, nmaps = 4096, 8
    g = si.healpix(2048)
    say("healpix 2048 lmax 4096: fp64 and mixed (8 maps)")
    alm = torch.empty((nmaps, si.nalm(lmax, lmax)), dtype=torch.complex128, device="cuda")
    for i in range(nmaps):
        alm[i] = dev(si.powerlaw_alm(lmax, lmax, si.config_seed(5, i)))
    f64 = sht.alm2map(alm, g, lmax)
    a0 = host(alm[0])
    # ring 2038 has 8156 = 4 x 2039 pixels: a direct radix-2039 stage
    assert g.nphi[2038] == 4 * 2039
    rings = np.union1d(np.arange(0, g.nrings, 8), [1, 2038, 2047, 4095, 8189, 8190]).astype(np.int32)
    say(f"healpix 2048 lmax 4096: oracle alm2map on {len(rings)} rings")
    ref = oracle.alm2map(lmax, lmax, g, a0, rings=rings)
    m0 = host(f64[0])
    px = np.concatenate([np.arange(g.ofs[r], g.ofs[r] + g.nphi[r]) for r in rings])
    err = relrms(m0[px], ref[px])
    say(f"healpix 2048 lmax 4096 alm2map rel rms over {len(rings)} rings {err:.3e}")
    assert err <= 1e-12
    # per ring (as few as 4 pixels) the FP64 bar scales with the 4096 steps of
    # the recurrence: 3e-12 in the north; a southern ring is evaluated at the
    # mirrored northern colatitude, half an ulp of pi from its own, which
    # moves the 4-pixel rings at the south pole by ~1e-11 here
    for r in rings:
        sl = slice(g.ofs[r], g.ofs[r] + g.nphi[r])
        tol = 3e-12 if r < g.nrings // 2 else 4e-11
        assert relrms(m0[sl], ref[sl]) <= tol, (r, relrms(m0[sl], ref[sl]))
    noise = si.random_map(g, 2048)
    back_n = host(sht.map2alm(dev(noise), g, lmax))
    ms = np.union1d(np.arange(0, lmax + 1, 8), [1, 5, 4095, 4096]).astype(np.int32)
    say(f"healpix 2048 lmax 4096: oracle map2alm on {len(ms)} m")
    ref = oracle.map2alm(lmax, lmax, g, noise, ms=ms)
    ix = np.concatenate([si.alm_index(np.arange(m, lmax + 1), m, lmax) for m in ms])
    err = relrms(back_n[ix], ref[ix])
    say(f"healpix 2048 lmax 4096 map2alm rel rms over {len(ms)} m {err:.3e}")
    assert err <= 1e-12
    for m in ms:
        idx = si.alm_index(np.arange(m, lmax + 1), m, lmax)
        assert relrms(back_n[idx], ref[idx]) <= 1e-11, (int(m), relrms(back_n[idx], ref[idx]))
    back64 = sht.map2alm(f64, g, lmax)
    mx = sht.alm2map(alm, g, lmax, flags=sht.SHT_MIXED)
    err_s = ((mx - f64).norm(dim=1) / f64.norm(dim=1)).cpu().numpy()
    back = sht.map2alm(f64, g, lmax, flags=sht.SHT_MIXED)
    err_a = ((back - back64).norm(dim=1) / back64.norm(dim=1)).cpu().numpy()
    say(f"lmax 4096 mixed rel rms: alm2map max {err_s.max():.3e}, map2alm max {err_a.max():.3e}")
    assert np.all(err_s <= 5e-7) and np.all(err_a <= MX_TOL), (err_s.max(), err_a.max())
