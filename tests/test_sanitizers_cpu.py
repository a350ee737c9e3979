"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

Two sanitized builds, each loaded in a subprocess with its sanitizer runtime
preloaded and driven through its C interface on seeded inputs:
- the oracle (gcc, -fsanitize=address,undefined): small transforms of every
  kind, extended-range Legendre values down to the deepest underflow;
- the transform library's host code (hipcc; the sanitizer flags apply to the
  host compilation only, after -Xarch_host): argument and geometry
  validation, ring pairing, workspace sizing, batch layout and the error
  paths, every call that needs no device.
Any report aborts the subprocess (no recovery), which fails the test.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _run(code, preload, tmp):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    # the interpreter itself is not instrumented: leak reports would be its own
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = ROOT
    script = os.path.join(tmp, "drive.py")
    with open(script, "w") as f:
        f.write(textwrap.dedent(code))
    r = subprocess.run([sys.executable, script], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stdout[-3000:], r.stderr[-6000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, r.stderr[-6000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not found")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    out = _run(f"""
        import numpy as np
        import oracle
        oracle._LIB = {lib!r}
        oracle._lib = None
        L = oracle._load()
        import sht_inputs as si
        oracle.set_threads(2)
        for g, lmax, mmax in ((si.healpix(4), 10, 7), (si.gauss_legendre(9, 17), 8, 8),
                              (si.gauss_legendre(1, 1), 0, 0)):
            a = si.uniform_alm(lmax, mmax, 3)
            m = oracle.alm2map(lmax, mmax, g, a)
            b = oracle.map2alm(lmax, mmax, g, m)
            d = oracle.delta_syn(lmax, mmax, g, a, rings=[0, g.nrings - 1])
            s = oracle.map2delta(mmax, g, m, ms=[0, mmax])
            oracle.delta2alm(lmax, mmax, g, oracle.map2delta(mmax, g, m), ms=[mmax])
            oracle.delta2map(mmax, g, oracle.delta_syn(lmax, mmax, g, a))
        mant, e = oracle.plm_ext(3000, 1500, 1e-3)
        v = oracle.plm(400, 7, 3.0)
        try:
            oracle.alm2map(-1, 0, si.healpix(1), np.zeros(1, complex))
        except ValueError:
            pass
        print("oracle ok", int(e.min()))
    """, f"{asan}:{ubsan}", str(tmp_path))
    assert "oracle ok" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    rt = _clang_asan_runtime()
    if not rt or not os.path.exists(HIPCC):
        pytest.skip("clang ASan runtime or hipcc not found")
    csrc = os.path.join(ROOT, "paper_1106_0159_amd", "csrc")
    from paper_1106_0159_amd import _build
    srcs = [os.path.join(csrc, s) for s in _build.SOURCES]
    lib = str(tmp_path / "libsht_asan.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), "-I" + csrc, *srcs, "-o", lib]
    subprocess.run(cmd, check=True, capture_output=True)
    out = _run(f"""
        import ctypes
        import numpy as np
        import paper_1106_0159_amd as sht
        sht.LIB_PATH = {lib!r}
        sht._lib = None
        L = sht.lib()
        import sht_inputs as si
        P = ctypes.c_void_p
        a, m, w = P(0x100000), P(0x200000), P(0x300000)
        big = 1 << 20
        geoms = [si.healpix(1), si.healpix(8), si.gauss_legendre(1, 1), si.gauss_legendre(33, 65),
                 si.subset_geometry(si.healpix(16), [5, 1, 60, 3, 40]),
                 si._pack(np.array([1e-3, 0.3, np.pi - 0.3, np.pi - 1e-3 + 5e-15]), np.array([7, 9, 9, 7], np.int32),
                          np.zeros(4), np.ones(4), "near")]
        for g in geoms:
            gh = sht.GeomHandle(g)
            for lmax, mmax in ((0, 0), (12, 5), (40, 40)):
                for f in (0, 1):
                    assert L.sht_workspace_bytes(lmax, mmax, gh.ref(), 3, f) > 0
            assert L.sht_workspace_bytes(4, 5, gh.ref(), 1, 0) == 0
            assert L.sht_alm2map(4, 4, gh.ref(), None, m, 1, w, big, 0, None) == sht.SHT_EINVAL
            assert L.sht_map2alm(4, 4, gh.ref(), m, a, 1, None, big, 0, None) == sht.SHT_EWORKSPACE
            assert L.sht_prepare(4, 4, gh.ref(), 8, None) == sht.SHT_EUNSUPPORTED
            assert sht.ring_slots(g.theta) >= (g.nrings + 1) // 2
        # overlapping and unordered ring offsets, NaN colatitudes
        g = si.healpix(4)
        bad = sht.GeomHandle(si._pack(g.theta, g.nphi, g.phi0, g.weight, "x"))
        bad.ofs[:] = bad.ofs[::-1].copy()
        assert L.sht_workspace_bytes(8, 8, bad.ref(), 1, 0) > 0  # any order, no overlap
        bad.ofs[1] = bad.ofs[0]
        assert L.sht_workspace_bytes(8, 8, bad.ref(), 1, 0) == 0
        nan = sht.GeomHandle(g)
        nan.theta[3] = np.nan
        assert L.sht_workspace_bytes(8, 8, nan.ref(), 1, 0) == 0
        # batches: sizing and validation of every request
        reqs = (sht._Request * 3)()
        gs = [sht.GeomHandle(si.gauss_legendre(9, 17)), sht.GeomHandle(si.healpix(4)),
              sht.GeomHandle(si.healpix(2), with_weight=False)]
        for i, (k, lm, tile) in enumerate(((0, 8, 0), (1, 8, 17), (0, 4, 4))):
            reqs[i] = sht._Request(k, lm, lm, ctypes.pointer(gs[i].c), 0x1000 * (i + 1), 0x9000 * (i + 1), tile)
        assert L.sht_batch_workspace_bytes(3, reqs, 0) > 0
        reqs[1].tile = 3
        assert L.sht_batch_workspace_bytes(3, reqs, 0) == 0
        reqs[1].tile = 0
        reqs[2].kind = 1  # analysis without weights
        assert L.sht_batch_workspace_bytes(3, reqs, 0) == 0
        h = P()
        assert L.sht_batch_create(3, reqs, None, 0, 0, None, ctypes.byref(h)) == sht.SHT_EINVAL
        for code in range(-7, 2):
            assert L.sht_strerror(code)
        assert L.sht_plan_cache_limits(3, 5) == 0 and L.sht_plan_cache_limits(8, 32) == 0
        assert L.sht_plan_cache_bytes() == 0
        print("library ok")
    """, rt, str(tmp_path))
    assert "library ok" in out
