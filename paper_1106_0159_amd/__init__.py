"""Python binding of libsht.so: argument marshalling only.

Every step of the transforms runs in the HIP library; torch is used for
device memory and the current stream.  If libsht.so has not been built the
import of the binding functions raises immediately: there is no CPU path.

Geometry objects are anything with numpy attributes ``theta`` (float64),
``nphi`` (int32), ``phi0`` (float64), ``weight`` (float64) and ``ofs``
(int64) per ring, e.g. ``sht_inputs.Geometry``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsht.so")

SHT_OK, SHT_EINVAL, SHT_EWORKSPACE, SHT_EDEVICE, SHT_ENOMEM, SHT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SHT_ENOPLAN = -6
SHT_MIXED = 1  # flag: FP32 matrix-core Legendre contraction (include/sht.h)
SHT_DELTA_MAP_MINOR = 2  # flag: stage-call Delta laid out [nrings][mmax+1][nmaps]
SHT_PIN = 4  # sht_prepare flag: keep the plan's tables until sht_unpin
SHT_MIXED_FP64_SUMS = 8  # with SHT_MIXED: synthesis block sums added in FP64
SHT_MIXED_SPLIT_BF16 = 16  # with SHT_MIXED, synthesis only: three-way bf16 split products

EXPORTS = ("sht_workspace_bytes", "sht_alm2map", "sht_map2alm", "sht_alm2delta", "sht_delta2map",
           "sht_map2delta", "sht_delta2alm", "sht_strerror", "sht_shutdown",
           "sht_prepare", "sht_unpin", "sht_plan_cache_limits", "sht_plan_cache_bytes",
           "sht_batch_workspace_bytes", "sht_batch_create", "sht_batch_run",
           "sht_batch_destroy", "sht_alm2map_noalloc")
SHT_ALM2MAP, SHT_MAP2ALM = 0, 1  # sht_request.kind


class ShtError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {lib().sht_strerror(code).decode()} (status {code})")
        self.code = code


class _Geom(ctypes.Structure):
    _fields_ = [("nrings", ctypes.c_int32), ("theta", ctypes.c_void_p), ("nphi", ctypes.c_void_p),
                ("phi0", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("ofs", ctypes.c_void_p)]


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("lmax", ctypes.c_int32), ("mmax", ctypes.c_int32),
                ("geom", ctypes.POINTER(_Geom)), ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("tile", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsht.so (raises if it is missing: the GPU library is required)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_1106_0159_amd/_build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, I, U, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_size_t
        GP = ctypes.POINTER(_Geom)
        L.sht_workspace_bytes.restype = S
        L.sht_workspace_bytes.argtypes = [I, I, GP, I, U]
        for name in ("sht_alm2map", "sht_map2alm", "sht_alm2delta"):
            f = getattr(L, name)
            f.restype = I
            f.argtypes = [I, I, GP, P, P, I, P, S, U, P]
        for name in ("sht_delta2map", "sht_map2delta"):
            f = getattr(L, name)
            f.restype = I
            f.argtypes = [I, GP, P, P, I, U, P]
        L.sht_delta2alm.restype = I
        L.sht_delta2alm.argtypes = [I, I, GP, P, P, I, P, S, U, P]
        L.sht_strerror.restype = ctypes.c_char_p
        L.sht_strerror.argtypes = [I]
        L.sht_shutdown.restype = None
        L.sht_shutdown.argtypes = []
        L.sht_prepare.restype = I
        L.sht_prepare.argtypes = [I, I, GP, U, P]
        L.sht_unpin.restype = I
        L.sht_unpin.argtypes = [I, I, GP]
        RP = ctypes.POINTER(_Request)
        L.sht_batch_workspace_bytes.restype = S
        L.sht_batch_workspace_bytes.argtypes = [I, RP, U]
        L.sht_batch_create.restype = I
        L.sht_batch_create.argtypes = [I, RP, P, S, U, P, ctypes.POINTER(P)]
        L.sht_batch_run.restype = I
        L.sht_batch_run.argtypes = [P, P]
        L.sht_batch_destroy.restype = None
        L.sht_batch_destroy.argtypes = [P]
        L.sht_alm2map_noalloc.restype = I
        L.sht_alm2map_noalloc.argtypes = [I, I, GP, P, P, I, U, P]
        L.sht_plan_cache_limits.restype = I
        L.sht_plan_cache_limits.argtypes = [I, I]
        L.sht_plan_cache_bytes.restype = S
        L.sht_plan_cache_bytes.argtypes = []
        _lib = L
    return _lib


class GeomHandle:
    """Keeps contiguous host copies of a geometry alive for ctypes."""

    def __init__(self, g, with_weight: bool = True):
        self.theta = np.ascontiguousarray(g.theta, dtype=np.float64)
        self.nphi = np.ascontiguousarray(g.nphi, dtype=np.int32)
        self.phi0 = np.ascontiguousarray(g.phi0, dtype=np.float64)
        w = getattr(g, "weight", None)
        self.weight = None if (w is None or not with_weight) else np.ascontiguousarray(w, dtype=np.float64)
        o = getattr(g, "ofs", None)
        self.ofs = None if o is None else np.ascontiguousarray(o, dtype=np.int64)
        self.nrings = int(self.theta.shape[0])
        self.npix = int(np.max(self.ofs + self.nphi)) if self.ofs is not None else int(self.nphi.sum())
        # rings never overlap (the library rejects that), so when their pixel
        # counts add up to npix every pixel of a synthesised map is written
        self.covers_all = int(self.nphi.sum()) == self.npix
        ptr = lambda a: None if a is None else a.ctypes.data
        self.c = _Geom(self.nrings, ptr(self.theta), ptr(self.nphi), ptr(self.phi0), ptr(self.weight),
                       ptr(self.ofs))

    def ref(self):
        return ctypes.byref(self.c)


def nalm(lmax: int, mmax: int) -> int:
    return (mmax + 1) * (2 * lmax + 2 - mmax) // 2


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc: int, what: str):
    if rc != SHT_OK:
        raise ShtError(rc, what)


def _gh(geom, with_weight=True) -> GeomHandle:
    return geom if isinstance(geom, GeomHandle) else GeomHandle(geom, with_weight)


def workspace_bytes(lmax: int, mmax: int, geom, nmaps: int = 1, flags: int = 0) -> int:
    g = _gh(geom)
    return int(lib().sht_workspace_bytes(lmax, mmax, g.ref(), nmaps, flags))


def workspace(lmax: int, mmax: int, geom, nmaps: int = 1, device="cuda", flags: int = 0):
    torch = _torch()
    n = workspace_bytes(lmax, mmax, geom, nmaps, flags)
    if n == 0:
        raise ShtError(SHT_EINVAL, "sht_workspace_bytes")
    return torch.empty(n, dtype=torch.uint8, device=device)


def _nmaps_of(t, per):
    n = t.numel() // per
    if n * per != t.numel() or n < 1:
        raise ValueError(f"tensor of {t.numel()} elements is not a whole number of {per}-element maps")
    return n


def alm2map(alm, geom, lmax: int, mmax: int | None = None, out=None, ws=None, stream=None, flags: int = 0):
    """Synthesis.  alm: complex128 CUDA tensor [..., nalm]; returns float64 [..., npix]."""
    torch = _torch()
    mmax = lmax if mmax is None else mmax
    g = _gh(geom, with_weight=False)
    na = nalm(lmax, mmax)
    nm = _nmaps_of(alm, na)
    if out is None:
        alloc = torch.empty if g.covers_all else torch.zeros
        out = alloc(alm.shape[:-1] + (g.npix,), dtype=torch.float64, device=alm.device)
    if ws is None:
        ws = workspace(lmax, mmax, g, nm, alm.device, flags)
    rc = lib().sht_alm2map(lmax, mmax, g.ref(), alm.data_ptr(), out.data_ptr(), nm, ws.data_ptr(),
                           ws.numel() * ws.element_size(), flags, _stream_ptr(stream))
    _check(rc, "sht_alm2map")
    return out


def map2alm(mp, geom, lmax: int, mmax: int | None = None, out=None, ws=None, stream=None, flags: int = 0):
    """Analysis.  mp: float64 CUDA tensor [..., npix]; returns complex128 [..., nalm]."""
    torch = _torch()
    mmax = lmax if mmax is None else mmax
    g = _gh(geom)
    nm = _nmaps_of(mp, g.npix)
    if out is None:
        out = torch.empty(mp.shape[:-1] + (nalm(lmax, mmax),), dtype=torch.complex128, device=mp.device)
    if ws is None:
        ws = workspace(lmax, mmax, g, nm, mp.device, flags)
    rc = lib().sht_map2alm(lmax, mmax, g.ref(), mp.data_ptr(), out.data_ptr(), nm, ws.data_ptr(),
                           ws.numel() * ws.element_size(), flags, _stream_ptr(stream))
    _check(rc, "sht_map2alm")
    return out


def alm2map_noalloc(alm, geom, lmax: int, mmax: int | None = None, out=None, stream=None, flags: int = 0):
    """sht_alm2map_noalloc (include/sht_noalloc.h): synthesis whose workspace
    is the library's fixed device scratch array.  The plan of (lmax, mmax,
    geom) must be prepared and pinned first (prepare(..., pin=True)) with the
    same geometry handle; pass `out` for a call that allocates nothing."""
    torch = _torch()
    mmax = lmax if mmax is None else mmax
    g = _gh(geom, with_weight=False)
    nm = _nmaps_of(alm, nalm(lmax, mmax))
    if out is None:
        alloc = torch.empty if g.covers_all else torch.zeros
        out = alloc(alm.shape[:-1] + (g.npix,), dtype=torch.float64, device=alm.device)
    rc = lib().sht_alm2map_noalloc(lmax, mmax, g.ref(), alm.data_ptr(), out.data_ptr(), nm, flags,
                                   _stream_ptr(stream))
    _check(rc, "sht_alm2map_noalloc")
    return out


def alm2delta(alm, geom, lmax: int, mmax: int | None = None, out=None, ws=None, stream=None, flags: int = 0):
    """Legendre synthesis stage: complex128 Delta [..., nrings, mmax+1]."""
    torch = _torch()
    mmax = lmax if mmax is None else mmax
    g = _gh(geom, with_weight=False)
    nm = _nmaps_of(alm, nalm(lmax, mmax))
    if out is None:
        shape = ((g.nrings, mmax + 1, nm) if flags & SHT_DELTA_MAP_MINOR
                 else alm.shape[:-1] + (g.nrings, mmax + 1))
        out = torch.empty(shape, dtype=torch.complex128, device=alm.device)
    if ws is None:
        ws = workspace(lmax, mmax, g, nm, alm.device, flags)
    rc = lib().sht_alm2delta(lmax, mmax, g.ref(), alm.data_ptr(), out.data_ptr(), nm, ws.data_ptr(),
                             ws.numel() * ws.element_size(), flags, _stream_ptr(stream))
    _check(rc, "sht_alm2delta")
    return out


def delta2map(delta, geom, mmax: int, out=None, stream=None, flags: int = 0):
    """Ring synthesis stage: float64 map [..., npix] from Delta [..., nrings, mmax+1]
    (or [nrings, mmax+1, nmaps] with SHT_DELTA_MAP_MINOR)."""
    torch = _torch()
    g = _gh(geom, with_weight=False)
    nm = _nmaps_of(delta, g.nrings * (mmax + 1))
    if out is None:
        shape = (nm, g.npix) if flags & SHT_DELTA_MAP_MINOR else delta.shape[:-2] + (g.npix,)
        alloc = torch.empty if g.covers_all else torch.zeros
        out = alloc(shape, dtype=torch.float64, device=delta.device)
    rc = lib().sht_delta2map(mmax, g.ref(), delta.data_ptr(), out.data_ptr(), nm, flags, _stream_ptr(stream))
    _check(rc, "sht_delta2map")
    return out


def map2delta(mp, geom, mmax: int, out=None, stream=None, flags: int = 0):
    """Ring analysis stage: Delta^S [..., nrings, mmax+1] (or [nrings, mmax+1, nmaps]
    with SHT_DELTA_MAP_MINOR) from a float64 map."""
    torch = _torch()
    g = _gh(geom)
    nm = _nmaps_of(mp, g.npix)
    if out is None:
        shape = ((g.nrings, mmax + 1, nm) if flags & SHT_DELTA_MAP_MINOR
                 else mp.shape[:-1] + (g.nrings, mmax + 1))
        out = torch.empty(shape, dtype=torch.complex128, device=mp.device)
    rc = lib().sht_map2delta(mmax, g.ref(), mp.data_ptr(), out.data_ptr(), nm, flags, _stream_ptr(stream))
    _check(rc, "sht_map2delta")
    return out


def delta2alm(delta, geom, lmax: int, mmax: int | None = None, out=None, ws=None, stream=None, flags: int = 0):
    """Legendre analysis stage: a_lm [..., nalm] from Delta^S [..., nrings, mmax+1]."""
    torch = _torch()
    mmax = lmax if mmax is None else mmax
    g = _gh(geom, with_weight=False)
    nm = _nmaps_of(delta, g.nrings * (mmax + 1))
    if out is None:
        shape = (nm,) if flags & SHT_DELTA_MAP_MINOR else delta.shape[:-2]
        out = torch.empty(shape + (nalm(lmax, mmax),), dtype=torch.complex128, device=delta.device)
    if ws is None:
        ws = workspace(lmax, mmax, g, nm, delta.device, flags)
    rc = lib().sht_delta2alm(lmax, mmax, g.ref(), delta.data_ptr(), out.data_ptr(), nm, ws.data_ptr(),
                             ws.numel() * ws.element_size(), flags, _stream_ptr(stream))
    _check(rc, "sht_delta2alm")
    return out


def prepare(geom, lmax: int, mmax: int | None = None, stream=None, flags: int = 0, pin: bool = False) -> None:
    """Build and keep resident the plan tables of (lmax, mmax, geom); returns
    once the start table's kernel has completed.  pin=True adds a pin (no
    eviction until unpin())."""
    mmax = lmax if mmax is None else mmax
    f = flags | (SHT_PIN if pin else 0)
    _check(lib().sht_prepare(lmax, mmax, _gh(geom).ref(), f, _stream_ptr(stream)), "sht_prepare")


def unpin(geom, lmax: int, mmax: int | None = None) -> None:
    """Remove one pin that prepare(..., pin=True) put on these plan tables."""
    mmax = lmax if mmax is None else mmax
    _check(lib().sht_unpin(lmax, mmax, _gh(geom).ref()), "sht_unpin")


def plan_cache_limits(max_coef_tables: int, max_geom_plans: int) -> None:
    _check(lib().sht_plan_cache_limits(max_coef_tables, max_geom_plans), "sht_plan_cache_limits")


def plan_cache_bytes() -> int:
    return int(lib().sht_plan_cache_bytes())


def ring_slots(theta) -> int:
    """Ring slots of a geometry as the library forms them (mirror pairs, with
    |theta + theta' - pi| <= 2^-50 summed exactly, plus unpaired rings)."""
    th = sorted(float(t) for t in np.asarray(theta))
    pi_l = np.longdouble("3.14159265358979323846264338327950288")
    i, j, n = 0, len(th) - 1, 0
    while i <= j:
        if i == j:
            return n + 1
        d = float((np.longdouble(th[i]) + np.longdouble(th[j])) - pi_l)
        if abs(d) <= 2.0 ** -50:
            i, j = i + 1, j - 1
        elif d < 0:
            i += 1
        else:
            j -= 1
        n += 1
    return n


class Batch:
    """An uneven batch (sht_batch_*): transforms of any lmax, geometry and
    direction whose Legendre stage runs in one persistent launch.

    requests: list of (kind, lmax, geom, input tensor, output tensor[, tile])
    with kind "alm2map" or "map2alm", one map each.  Outputs may be None (they
    are allocated).  Inputs, outputs and the workspace are bound to the batch:
    every run() reads the inputs and writes the outputs."""

    def __init__(self, requests, device="cuda", stream=None, tiles=None):
        """tiles: None (the library's choice), "auto" (the autotuner's table,
        autotune.TABLE_PATH) or a table dict; a tile given in a request wins."""
        torch = _torch()
        if tiles == "auto":
            from . import autotune
            tiles = autotune.load()
        self.geoms, self.inputs, self.outputs, self.kinds = [], [], [], []
        arr = (_Request * len(requests))()
        for i, rq in enumerate(requests):
            kind, lmax, geom, x, y = rq[:5]
            tile = rq[5] if len(rq) > 5 else 0
            if not tile and tiles:
                from . import autotune
                tile = autotune.choose(tiles, kind, lmax, ring_slots(_gh(geom).theta))
            k = {"alm2map": SHT_ALM2MAP, "map2alm": SHT_MAP2ALM}[kind]
            g = _gh(geom, with_weight=True)
            if y is None:
                if k == SHT_ALM2MAP:
                    alloc = torch.empty if g.covers_all else torch.zeros
                    y = alloc(g.npix, dtype=torch.float64, device=device)
                else:
                    y = torch.empty(nalm(lmax, lmax), dtype=torch.complex128, device=device)
            self.geoms.append(g)
            self.inputs.append(x)
            self.outputs.append(y)
            self.kinds.append(kind)
            arr[i] = _Request(k, lmax, lmax, ctypes.pointer(g.c), x.data_ptr(), y.data_ptr(), tile)
        self._reqs = arr
        n = int(lib().sht_batch_workspace_bytes(len(requests), arr, 0))
        if n == 0:
            raise ShtError(SHT_EINVAL, "sht_batch_workspace_bytes")
        self.workspace = torch.empty(n, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib().sht_batch_create(len(requests), arr, self.workspace.data_ptr(), n, 0, _stream_ptr(stream),
                                      ctypes.byref(h)), "sht_batch_create")
        self._h = h

    def run(self, stream=None) -> None:
        _check(lib().sht_batch_run(self._h, _stream_ptr(stream)), "sht_batch_run")

    def close(self) -> None:
        """Free the batch (after the device has finished every run of it)."""
        if getattr(self, "_h", None) is not None and self._h.value:
            _torch().cuda.synchronize()
            lib().sht_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shutdown() -> None:
    lib().sht_shutdown()
