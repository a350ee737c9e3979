"""ctypes binding of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product library never loads it.

Functions take and return numpy arrays; a_lm are complex128 m-major packed,
maps float64, Delta arrays complex128 (see ``oracle.h``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BUILD_CMD = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC",
             "-shared", "-Wall", "-Wextra", "-o", _LIB, _SRC, "-lm"]


def build() -> str:
    """Compile liboracle.so (always)."""
    subprocess.run(BUILD_CMD, check=True, cwd=_HERE)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < max(
                os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        sig = {
            "oracle_set_threads": (None, [I]),
            "oracle_get_threads": (I, []),
            "oracle_plm_ext": (I, [I, I, D, P, P]),
            "oracle_plm": (I, [I, I, D, P]),
            "oracle_delta_syn": (I, [I, I, I, P, P, I, P, P]),
            "oracle_delta2map": (I, [I, I, P, P, P, P, I, P, P]),
            "oracle_alm2map": (I, [I, I, I, P, P, P, P, P, I, P, P]),
            "oracle_map2delta": (I, [I, I, P, P, P, P, P, I, P, P]),
            "oracle_delta2alm": (I, [I, I, I, P, P, I, P, P]),
            "oracle_map2alm": (I, [I, I, I, P, P, P, P, P, P, I, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _sel(sel):
    if sel is None:
        return None, 0
    s = np.ascontiguousarray(sel, dtype=np.int32)
    return s, int(s.shape[0])


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments")


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def plm_ext(lmax: int, m: int, theta: float):
    """lambda_lm(cos theta), l = m..lmax, as (mantissa, base-2 exponent)."""
    n = lmax - m + 1
    mant = np.zeros(n)
    e = np.zeros(n, dtype=np.int32)
    _check(_load().oracle_plm_ext(lmax, m, float(theta), _p(mant), _p(e)), "plm_ext")
    return mant, e


def plm(lmax: int, m: int, theta: float) -> np.ndarray:
    out = np.zeros(lmax - m + 1)
    _check(_load().oracle_plm(lmax, m, float(theta), _p(out)), "plm")
    return out


def delta_syn(lmax, mmax, geom, alm, rings=None) -> np.ndarray:
    th = _f64(geom.theta)
    a = _c128(alm)
    sel, ns = _sel(rings)
    cnt = ns if sel is not None else geom.nrings
    out = np.zeros((cnt, mmax + 1), dtype=np.complex128)
    _check(_load().oracle_delta_syn(lmax, mmax, geom.nrings, _p(th), _p(a), ns, _p(sel), _p(out)),
           "delta_syn")
    return out


def delta2map(mmax, geom, delta, rings=None, out=None) -> np.ndarray:
    d = _c128(delta)
    sel, ns = _sel(rings)
    m = np.zeros(geom.npix) if out is None else out
    _check(_load().oracle_delta2map(mmax, geom.nrings, _p(geom.nphi), _p(geom.phi0), _p(geom.ofs),
                                    _p(d), ns, _p(sel), _p(m)), "delta2map")
    return m


def alm2map(lmax, mmax, geom, alm, rings=None) -> np.ndarray:
    """Map on all rings (rings=None) or only on the listed rings (others left 0)."""
    a = _c128(alm)
    sel, ns = _sel(rings)
    m = np.zeros(geom.npix)
    _check(_load().oracle_alm2map(lmax, mmax, geom.nrings, _p(geom.theta), _p(geom.nphi),
                                  _p(geom.phi0), _p(geom.ofs), _p(a), ns, _p(sel), _p(m)),
           "alm2map")
    return m


def map2delta(mmax, geom, mp, ms=None) -> np.ndarray:
    s = _f64(mp)
    sel, nm = _sel(ms)
    cnt = nm if sel is not None else mmax + 1
    out = np.zeros((geom.nrings, cnt), dtype=np.complex128)
    _check(_load().oracle_map2delta(mmax, geom.nrings, _p(geom.nphi), _p(geom.phi0),
                                    _p(geom.weight), _p(geom.ofs), _p(s), nm, _p(sel), _p(out)),
           "map2delta")
    return out


def delta2alm(lmax, mmax, geom, delta, ms=None, out=None) -> np.ndarray:
    d = _c128(delta)
    sel, nm = _sel(ms)
    from sht_inputs import nalm
    a = np.zeros(nalm(lmax, mmax), dtype=np.complex128) if out is None else out
    _check(_load().oracle_delta2alm(lmax, mmax, geom.nrings, _p(geom.theta), _p(d), nm, _p(sel),
                                    _p(a)), "delta2alm")
    return a


def map2alm(lmax, mmax, geom, mp, ms=None) -> np.ndarray:
    """a_lm for all m (ms=None) or only the listed m (other entries left 0)."""
    s = _f64(mp)
    sel, nm = _sel(ms)
    from sht_inputs import nalm
    a = np.zeros(nalm(lmax, mmax), dtype=np.complex128)
    _check(_load().oracle_map2alm(lmax, mmax, geom.nrings, _p(geom.theta), _p(geom.nphi),
                                  _p(geom.phi0), _p(geom.weight), _p(geom.ofs), _p(s), nm,
                                  _p(sel), _p(a)), "map2alm")
    return a
