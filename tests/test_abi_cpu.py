"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, sizes its workspace, and rejects invalid arguments on the host
before any device work is enqueued."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import sht_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))

sht = pytest.importorskip("paper_1106_0159_amd")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sht.LIB_PATH):
        pytest.skip("libsht.so not built")
    return sht.lib()


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sht_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(sht.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name
    # and the same names are visible to the dynamic linker
    nm = os.popen(f"nm -D --defined-only {sht.LIB_PATH}").read()
    for name in declared_functions():
        assert re.search(rf"\bT {name}$", nm, flags=re.M), name


def test_strerror_strings(L):
    for code in (0, -1, -2, -4, -5, 7):
        assert len(L.sht_strerror(code)) > 0
    assert L.sht_strerror(sht.SHT_EINVAL) == b"invalid argument"


def _ws(lmax, mmax, g, nmaps=1, flags=0):
    return sht.workspace_bytes(lmax, mmax, g, nmaps, flags)


def test_workspace_bytes_values_and_monotonic():
    g = si.healpix(8)
    lmax = 16
    na = si.nalm(lmax, lmax)
    r256 = lambda b: (b + 255) // 256 * 256
    # [Delta][aux]; 16 slots need one analysis group, so aux holds the scaled
    # a_lm and 32 padding entries that synthesis may read ahead
    pad = 32 * 16
    assert _ws(lmax, lmax, g) == r256(na * 16 + pad) + r256(g.nrings * (lmax + 1) * 16)
    assert _ws(lmax, lmax, g, 3) == r256(3 * na * 16 + pad) + r256(3 * g.nrings * (lmax + 1) * 16)
    # HEALPix nside=1024: 2048 slots fit one analysis workgroup; nside=2048:
    # 4096 slots -> two groups of 2048, whose partial a_lm fill aux
    na2 = si.nalm(64, 64)
    big = si.healpix(1024)
    assert _ws(64, 64, big) == r256(big.nrings * 65 * 16) + r256(na2 * 16 + pad)
    big = si.healpix(2048)
    assert _ws(64, 64, big) == r256(big.nrings * 65 * 16) + r256(2 * na2 * 16)
    prev = 0
    for l in range(0, 40, 3):
        cur = _ws(l, l, g)
        assert cur > prev
        prev = cur
    assert _ws(lmax, lmax, g) % 256 == 0


def test_workspace_bytes_mixed():
    """SHT_MIXED: aux holds FP32 tiles of c a_lm, [column group][l-block of
    column m][parity][16 NCF columns][16 k] floats, NCF = 1, 2, 4 for up to
    8, 16 and more maps (8 NCF maps per column group; NCF = 1 with FP64
    block sums and above lmax 2048; with the bf16 split the tiles hold three
    bf16 planes), kMxL = 32 l per block, or the FP64 c-scaled a_lm if
    larger."""
    g = si.healpix(8)
    r256 = lambda b: (b + 255) // 256 * 256
    delta = lambda lmax, n: r256(n * g.nrings * (lmax + 1) * 16)

    def tiles(lmax, nmaps, f64_sums=False, split=False):
        blocks = sum((lmax - m + 32) // 32 for m in range(lmax + 1))
        ncf = 1 if nmaps <= 8 else 2 if nmaps <= 16 else 4
        if lmax > 2048 or f64_sums:  # FP64 block sums: 8 maps per wave
            ncf = 1
        ncg = -(-nmaps // (8 * ncf))
        # split: three bf16 planes (6 bytes per entry) instead of FP32
        return ncg * blocks * 2 * (16 * ncf) * 16 * (6 if split else 4)

    # with SHT_MIXED either kernel set may run (the FP64 ones below 8 maps),
    # so aux holds the larger of the tiles and the c-scaled a_lm (+32 entries)
    def aux(lmax, nmaps, f64_sums=False, split=False):
        f64 = nmaps * (lmax + 1) * (lmax + 2) // 2 * 16 + 32 * 16
        return r256(max(tiles(lmax, nmaps, f64_sums, split), f64))

    for lmax, nmaps in [(16, 1), (16, 3), (16, 12), (16, 20), (16, 40), (70, 33), (0, 1), (2048, 40), (2049, 40)]:
        assert _ws(lmax, lmax, g, nmaps, sht.SHT_MIXED) == delta(lmax, nmaps) + aux(lmax, nmaps), (lmax, nmaps)
        assert (_ws(lmax, lmax, g, nmaps, sht.SHT_MIXED | sht.SHT_MIXED_FP64_SUMS) ==
                delta(lmax, nmaps) + aux(lmax, nmaps, True)), (lmax, nmaps)
        assert (_ws(lmax, lmax, g, nmaps, sht.SHT_MIXED | sht.SHT_MIXED_SPLIT_BF16) ==
                delta(lmax, nmaps) + aux(lmax, nmaps, split=True)), (lmax, nmaps)
        assert (_ws(lmax, lmax, g, nmaps, sht.SHT_MIXED | sht.SHT_MIXED_SPLIT_BF16 | sht.SHT_MIXED_FP64_SUMS) ==
                delta(lmax, nmaps) + aux(lmax, nmaps, True, True)), (lmax, nmaps)
    # the FP64-sums bit needs SHT_MIXED
    assert _ws(16, 16, g, 1, sht.SHT_MIXED_FP64_SUMS) == 0
    # the Delta layout flag does not change the workspace
    for nmaps in (1, 20):
        assert _ws(16, 16, g, nmaps, sht.SHT_MIXED | sht.SHT_DELTA_MAP_MINOR) == _ws(16, 16, g, nmaps, sht.SHT_MIXED)
        assert _ws(16, 16, g, nmaps, sht.SHT_DELTA_MAP_MINOR) == _ws(16, 16, g, nmaps)
    # lmax = 16: 17 columns of one block each; 20 maps -> one group of 32 maps (64 columns)
    assert tiles(16, 20) == 17 * 2 * 64 * 16 * 4


@pytest.mark.parametrize("args", [
    (-1, 0, 1, 0), (4, 5, 1, 0), (4, -1, 1, 0), (4, 4, 0, 0), (4, 4, 1, 1 << 3), (4, 4, 1, 1 << 4),
])
def test_workspace_bytes_invalid(args):
    lmax, mmax, nmaps, flags = args
    assert _ws(lmax, mmax, si.healpix(2), nmaps, flags) == 0


def _geom_variant(**kw):
    g = si.healpix(2)
    d = dict(theta=g.theta.copy(), nphi=g.nphi.copy(), phi0=g.phi0.copy(), weight=g.weight.copy(),
             ofs=g.ofs.copy())
    d.update(kw)
    return si.Geometry(d["theta"], d["nphi"], d["phi0"], d["weight"], d["ofs"])


BAD_GEOMS = {
    "theta_negative": lambda g: _geom_variant(theta=np.r_[-0.1, g.theta[1:]]),
    "theta_above_pi": lambda g: _geom_variant(theta=np.r_[g.theta[:-1], 3.2]),
    "theta_nan": lambda g: _geom_variant(theta=np.r_[np.nan, g.theta[1:]]),
    "nphi_zero": lambda g: _geom_variant(nphi=np.r_[0, g.nphi[1:]].astype(np.int32)),
    "phi0_inf": lambda g: _geom_variant(phi0=np.r_[np.inf, g.phi0[1:]]),
    "overlap": lambda g: _geom_variant(ofs=np.r_[0, 1, g.ofs[2:]].astype(np.int64)),
    "ofs_negative": lambda g: _geom_variant(ofs=np.r_[-4, g.ofs[1:]].astype(np.int64)),
}


@pytest.mark.parametrize("name", sorted(BAD_GEOMS))
def test_invalid_geometry_rejected_on_host(L, name):
    g = BAD_GEOMS[name](si.healpix(2))
    gh = sht.GeomHandle(g)
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first
    rc = L.sht_alm2map(4, 4, gh.ref(), fake, fake, 1, fake, 1 << 20, 0, None)
    assert rc == sht.SHT_EINVAL
    rc = L.sht_map2alm(4, 4, gh.ref(), fake, fake, 1, fake, 1 << 20, 0, None)
    assert rc == sht.SHT_EINVAL
    assert L.sht_workspace_bytes(4, 4, gh.ref(), 1, 0) == 0


def test_invalid_arguments_rejected_on_host(L):
    g = sht.GeomHandle(si.healpix(2))
    a = ctypes.c_void_p(0x100000)
    m = ctypes.c_void_p(0x200000)
    w = ctypes.c_void_p(0x300000)
    big = 1 << 20
    # sizes
    assert L.sht_alm2map(-1, 0, g.ref(), a, m, 1, w, big, 0, None) == sht.SHT_EINVAL
    assert L.sht_alm2map(4, 5, g.ref(), a, m, 1, w, big, 0, None) == sht.SHT_EINVAL
    assert L.sht_alm2map(4, 4, g.ref(), a, m, 0, w, big, 0, None) == sht.SHT_EINVAL
    # flags: unknown bits; the map-minor Delta layout needs SHT_MIXED in the Legendre stage calls
    assert L.sht_alm2map(4, 4, g.ref(), a, m, 1, w, big, 8, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_alm2map(4, 4, g.ref(), a, m, 1, w, big, sht.SHT_PIN, None) == sht.SHT_EUNSUPPORTED  # sht_prepare only
    assert L.sht_alm2map(4, 4, g.ref(), a, m, 1, w, big, 1 << 31, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_map2alm(4, 4, g.ref(), m, a, 1, w, big, sht.SHT_MIXED | 4, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_delta2alm(4, 4, g.ref(), m, a, 1, w, big, 8, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_delta2map(4, g.ref(), m, a, 1, 32, None) == sht.SHT_EUNSUPPORTED
    # the split-bf16 bit needs SHT_MIXED and is a synthesis variant (analysis calls reject it)
    sp = sht.SHT_MIXED | sht.SHT_MIXED_SPLIT_BF16
    assert L.sht_alm2map(4, 4, g.ref(), a, m, 1, w, big, sht.SHT_MIXED_SPLIT_BF16, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_alm2delta(4, 4, g.ref(), a, m, 1, w, big, sht.SHT_MIXED_SPLIT_BF16, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_map2alm(4, 4, g.ref(), m, a, 1, w, big, sp, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_delta2alm(4, 4, g.ref(), m, a, 1, w, big, sp, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_workspace_bytes(4, 4, g.ref(), 1, sht.SHT_MIXED_SPLIT_BF16) == 0
    assert L.sht_alm2delta(4, 4, g.ref(), a, m, 1, w, big, sht.SHT_DELTA_MAP_MINOR, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_delta2alm(4, 4, g.ref(), m, a, 1, w, big, sht.SHT_DELTA_MAP_MINOR, None) == sht.SHT_EUNSUPPORTED
    # null and misaligned pointers
    assert L.sht_alm2map(4, 4, g.ref(), None, m, 1, w, big, 0, None) == sht.SHT_EINVAL
    assert L.sht_alm2map(4, 4, g.ref(), a, None, 1, w, big, 0, None) == sht.SHT_EINVAL
    assert L.sht_alm2map(4, 4, g.ref(), ctypes.c_void_p(0x100008), m, 1, w, big, 0, None) == sht.SHT_EINVAL
    assert L.sht_alm2map(4, 4, None, a, m, 1, w, big, 0, None) == sht.SHT_EINVAL
    # workspace
    need = L.sht_workspace_bytes(4, 4, g.ref(), 1, 0)
    assert L.sht_alm2map(4, 4, g.ref(), a, m, 1, None, big, 0, None) == sht.SHT_EWORKSPACE
    assert L.sht_alm2map(4, 4, g.ref(), a, m, 1, w, need - 1, 0, None) == sht.SHT_EWORKSPACE
    assert L.sht_map2alm(4, 4, g.ref(), m, a, 1, w, 16, 0, None) == sht.SHT_EWORKSPACE
    # aliasing buffers
    assert L.sht_alm2map(4, 4, g.ref(), a, a, 1, w, big, 0, None) == sht.SHT_EINVAL
    assert L.sht_alm2map(4, 4, g.ref(), a, m, 1, a, big, 0, None) == sht.SHT_EINVAL
    # analysis needs weights
    nw = sht.GeomHandle(si.healpix(2), with_weight=False)
    assert L.sht_map2alm(4, 4, nw.ref(), m, a, 1, w, big, 0, None) == sht.SHT_EINVAL
    assert L.sht_map2delta(4, nw.ref(), m, a, 1, 0, None) == sht.SHT_EINVAL
    # stage entry points
    assert L.sht_delta2alm(4, 5, g.ref(), a, m, 1, w, big, 0, None) == sht.SHT_EINVAL
    assert L.sht_delta2alm(4, 4, g.ref(), a, m, 1, None, big, 0, None) == sht.SHT_EWORKSPACE
    assert L.sht_delta2map(4, g.ref(), None, m, 1, 0, None) == sht.SHT_EINVAL
    assert L.sht_alm2delta(4, 4, g.ref(), a, m, 1, w, 8, 0, None) == sht.SHT_EWORKSPACE


def test_plan_calls_checked_on_host(L):
    """sht_prepare and sht_unpin validate their arguments before any device
    call."""
    g = sht.GeomHandle(si.healpix(2))
    assert L.sht_prepare(4, 4, g.ref(), 8, None) == sht.SHT_EUNSUPPORTED
    assert L.sht_prepare(4, 5, g.ref(), sht.SHT_PIN, None) == sht.SHT_EINVAL
    assert L.sht_unpin(4, 5, g.ref()) == sht.SHT_EINVAL
    assert L.sht_unpin(4, 4, None) == sht.SHT_EINVAL
    assert L.sht_strerror(sht.SHT_ENOPLAN).startswith(b"plan tables not resident")


def test_probe_library_is_separate_and_checks_arguments():
    """The throughput probes live in their own benchmark-only library
    (libsht_probe.so, probe/sht_probe.h), not in the transform library.  Flop
    counts: 256 threads per workgroup, 8 chains; FP64 FMA 2 flops per lane
    and step, matrix instructions 2*16*16*K per wave and step (K = 4 for FP32,
    32 for BF16); the interleaved probe is the sum of its two streams."""
    from paper_1106_0159_amd import probe
    if not os.path.exists(probe.LIB_PATH):
        pytest.skip("libsht_probe.so not built")
    if os.path.exists(sht.LIB_PATH):
        nm = os.popen(f"nm -D --defined-only {sht.LIB_PATH}").read()
        assert "sht_probe" not in nm
    P = probe.lib()
    blocks, iters = 3, 5
    assert P.sht_probe_flops(0, blocks, iters) == blocks * 256 * iters * 8 * 2
    assert P.sht_probe_flops(1, blocks, iters) == blocks * 4 * iters * 8 * 2 * 16 * 16 * 4
    assert P.sht_probe_flops(2, blocks, iters) == blocks * 4 * iters * 8 * 2 * 16 * 16 * 32
    # kinds 1 and 0 interleaved: kind 1 at iters plus kind 0 at 8 x iters
    assert P.sht_probe_flops(3, blocks, iters) == (P.sht_probe_flops(1, blocks, iters)
                                                   + P.sht_probe_flops(0, blocks, 8 * iters))
    for kind, b, it in [(4, 1, 1), (-1, 1, 1), (0, 0, 1), (0, 1, 0)]:
        assert P.sht_probe_flops(kind, b, it) == 0.0
    # rejected on the host, before any device call
    assert P.sht_probe_run(0, 1, 1, None, None) == -1
    assert P.sht_probe_run(7, 1, 1, ctypes.c_void_p(0x1000), None) == -1
