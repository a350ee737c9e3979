"""Seeded synthetic inputs for the spherical harmonic transforms.

This module is shared by the CPU oracle's tests and by the GPU path's tests
and benchmark.  It builds *inputs only*: ring geometries (Gauss-Legendre and
HEALPix ring layouts), the packed a_lm index convention and seeded random
a_lm.  None of the transform arithmetic (Legendre recurrence, seeds,
Fourier sums) lives here.

Geometry follows the iso-latitude ring constraints of the paper (Sec. 2.2):
every ring has one colatitude theta, ``nphi`` equidistant pixels starting at
longitude ``phi0``, one per-pixel quadrature weight, and a pixel offset in
the map.  Rings are ordered by increasing theta, pixels by increasing j
(phi_j = phi0 + 2*pi*j/nphi).

The a_lm array is complex128, m-major packed over m >= 0 (real maps only
need m >= 0, Sec. 2.1 eq. YlmDef and the conjugate symmetry stated beside
it): index(l, m) = m*(2*lmax + 1 - m)/2 + l for m <= l <= lmax.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

__all__ = [
    "Geometry", "gauss_legendre", "healpix", "nalm", "alm_index",
    "powerlaw_alm", "uniform_alm", "random_map", "config_seed", "subset_geometry", "serving_trace",
]


@dataclasses.dataclass
class Geometry:
    """Iso-latitude ring geometry (host arrays)."""
    theta: np.ndarray    # float64 [nrings], colatitude in [0, pi]
    nphi: np.ndarray     # int32   [nrings]
    phi0: np.ndarray     # float64 [nrings]
    weight: np.ndarray   # float64 [nrings], per-pixel quadrature weight
    ofs: np.ndarray      # int64   [nrings], first pixel of each ring in the map
    name: str = "custom"

    @property
    def nrings(self) -> int:
        return int(self.theta.shape[0])

    @property
    def npix(self) -> int:
        return int(self.ofs[-1] + self.nphi[-1]) if self.nrings else 0

    def validate(self) -> None:
        assert self.theta.dtype == np.float64 and self.phi0.dtype == np.float64
        assert self.nphi.dtype == np.int32 and self.ofs.dtype == np.int64
        assert self.weight.dtype == np.float64
        n = self.nrings
        for a in (self.nphi, self.phi0, self.weight, self.ofs):
            assert a.shape == (n,)


def _pack(theta, nphi, phi0, weight, name) -> Geometry:
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    nphi = np.ascontiguousarray(nphi, dtype=np.int32)
    phi0 = np.ascontiguousarray(phi0, dtype=np.float64)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    ofs = np.zeros(theta.shape[0], dtype=np.int64)
    if theta.shape[0] > 1:
        ofs[1:] = np.cumsum(nphi[:-1].astype(np.int64))
    g = Geometry(theta, nphi, phi0, weight, ofs, name)
    g.validate()
    return g


def _mirror(theta_n):
    """Colatitudes of the mirror rings: pi - theta computed in long double, rounded once."""
    return (_PI_L - np.asarray(theta_n, dtype=np.longdouble)).astype(np.float64)


_PI_L = np.longdouble("3.14159265358979323846264338327950288")


@functools.lru_cache(maxsize=16)
def _gl_north(n: int):
    """Positive Gauss-Legendre nodes (descending) and weights, long-double Newton.

    numpy's ``leggauss`` supplies the starting nodes; its weights lose about
    eight digits near the ends for n ~ 1000, so nodes are polished by Newton
    steps on P_n in long double and weights recomputed from
    w = 2 / ((1 - x^2) P_n'(x)^2).
    """
    x0, _ = np.polynomial.legendre.leggauss(n)
    xl = np.sort(x0[x0 > 0])[::-1].astype(np.longdouble)

    def pn(x):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = n * (x * p1 - p0) / (x * x - 1)
        return p1, dp

    for _ in range(3):
        p, dp = pn(xl)
        xl = xl - p / dp
    _, dp = pn(xl)
    wl = 2 / ((1 - xl * xl) * dp * dp)
    return np.arccos(xl).astype(np.float64), wl.astype(np.float64)


def gauss_legendre(nrings: int, nphi: int, phi0: float = 0.0) -> Geometry:
    """Gauss-Legendre rings: nodes cos(theta_r) of P_nrings, ``nphi`` pixels each.

    The per-pixel weight is 2*pi*w_GL/nphi so that sum_pixels weight = 4*pi.
    Southern rings are mirrors theta_s = pi - theta_n of the northern ones
    with the same weight; an odd ring count adds the equator ring.
    """
    th_n, w_n = _gl_north(nrings)
    half = nrings // 2
    theta = np.empty(nrings)
    wts = np.empty(nrings)
    theta[:half] = th_n
    wts[:half] = w_n
    theta[nrings - half:] = _mirror(th_n)[::-1]
    wts[nrings - half:] = w_n[::-1]
    if nrings % 2:
        theta[half] = math.pi / 2
        # weight of the zero node: 2 / P_n'(0)^2 from the normalisation sum
        wts[half] = 2.0 - 2.0 * float(np.sum(w_n.astype(np.longdouble)))
    return _pack(theta, np.full(nrings, nphi), np.full(nrings, phi0),
                 wts * (2.0 * math.pi / nphi), f"gl_{nrings}x{nphi}")


def healpix(nside: int) -> Geometry:
    """HEALPix ring scheme (Gorski et al. 2005): 4*nside-1 rings, 12*nside^2 pixels.

    North cap i = 1..nside-1: 1 - z = i^2/(3 nside^2), nphi = 4i, phi0 = pi/(4i).
    Belt i = nside..3 nside: z = (4 nside - 2i)/(3 nside), nphi = 4 nside,
    phi0 = pi/(2 nside) * (1 - s/2), s = (i - nside + 1) mod 2.
    South cap mirrored (theta -> pi - theta).  Equal-area weight 4*pi/npix.
    theta in the caps is taken from the exact 1 - z via a half-angle formula.
    """
    nr = 4 * nside - 1
    theta = np.empty(nr)
    nphi = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    for i in range(1, 2 * nside + 1):                   # northern half + equator
        r = i - 1
        if i < nside:
            # sin(theta/2) = sqrt((1-z)/2) = i / (sqrt(6) nside)
            theta[r] = 2.0 * math.asin(i / (math.sqrt(6.0) * nside))
            nphi[r] = 4 * i
            phi0[r] = math.pi / (4 * i)
        else:
            z = (4 * nside - 2 * i) / (3.0 * nside)
            theta[r] = math.acos(z)
            nphi[r] = 4 * nside
            s = (i - nside + 1) % 2
            phi0[r] = math.pi / (2 * nside) * (1.0 - 0.5 * s)
    for i in range(2 * nside + 1, 4 * nside):           # southern half
        r = i - 1
        m = 4 * nside - i                               # mirrored northern ring index
        theta[r] = float(_mirror(np.array([theta[m - 1]]))[0])
        if i > 3 * nside:
            nphi[r] = nphi[m - 1]
            phi0[r] = phi0[m - 1]
        else:
            nphi[r] = 4 * nside
            s = (i - nside + 1) % 2
            phi0[r] = math.pi / (2 * nside) * (1.0 - 0.5 * s)
    npix = 12 * nside * nside
    return _pack(theta, nphi, phi0, np.full(nr, 4.0 * math.pi / npix), f"healpix_{nside}")


def subset_geometry(g: Geometry, rings) -> Geometry:
    """Keep only the listed rings (re-packed, offsets recomputed)."""
    idx = np.asarray(rings, dtype=np.int64)
    return _pack(g.theta[idx], g.nphi[idx], g.phi0[idx], g.weight[idx], g.name + "_sub")


# ---------------------------------------------------------------- a_lm layout
def nalm(lmax: int, mmax: int) -> int:
    """Number of stored (l, m) pairs, m in [0, mmax], l in [m, lmax]."""
    return (mmax + 1) * (2 * lmax + 2 - mmax) // 2


def alm_index(l, m, lmax: int):
    """Packed m-major index of (l, m)."""
    return m * (2 * lmax + 1 - m) // 2 + l


def _lm_arrays(lmax: int, mmax: int):
    ls, ms = [], []
    for m in range(mmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


def config_seed(config: int, map_index: int = 0) -> int:
    return 11060000 + 1000 * config + map_index


def powerlaw_alm(lmax: int, mmax: int, seed: int) -> np.ndarray:
    """Power-law a_lm: C_l = 1/(l(l+1)) for l >= 2, C_0 = C_1 = 0.

    Re, Im ~ N(0, C_l/2) for m > 0; a_l0 real ~ N(0, C_l).
    """
    rng = np.random.default_rng(seed)
    l, m = _lm_arrays(lmax, mmax)
    cl = np.zeros(l.shape[0])
    big = l >= 2
    cl[big] = 1.0 / (l[big] * (l[big] + 1.0))
    re = rng.standard_normal(l.shape[0])
    im = rng.standard_normal(l.shape[0])
    sd = np.sqrt(cl / 2.0)
    a = (re * sd + 1j * im * sd).astype(np.complex128)
    z = m == 0
    a[z] = re[z] * np.sqrt(cl[z])
    return a


def uniform_alm(lmax: int, mmax: int, seed: int) -> np.ndarray:
    """The paper's accuracy protocol input (Sec. 5): Re, Im uniform in (-1, 1); Im a_l0 = 0."""
    rng = np.random.default_rng(seed)
    n = nalm(lmax, mmax)
    a = rng.uniform(-1.0, 1.0, n) + 1j * rng.uniform(-1.0, 1.0, n)
    a[: lmax + 1] = a[: lmax + 1].real
    return a.astype(np.complex128)


def random_map(g: Geometry, seed: int) -> np.ndarray:
    """A white-noise real map on geometry g (for adjointness and analysis tests)."""
    return np.random.default_rng(seed).standard_normal(g.npix)


def serving_trace(n: int, seed: int, lmin: int = 64, lmax_hi: int = 4096):
    """A serving workload of n requests: lmax = 2*round(exp(U[ln lmin, ln lmax_hi])/2)
    (even, for a HEALPix grid with nside = lmax/2), each request alm2map or
    map2alm with probability 1/2, and Poisson arrival times of unit rate
    (divide by the offered rate), the first at t = 0.

    Returns (lmax int64 [n], kinds str [n], arrival float64 [n])."""
    rng = np.random.default_rng(seed)
    lm = 2 * np.round(np.exp(rng.uniform(np.log(lmin), np.log(lmax_hi), n)) / 2).astype(np.int64)
    kinds = np.where(rng.random(n) < 0.5, "alm2map", "map2alm")
    gaps = rng.exponential(1.0, n)
    return lm, kinds, np.cumsum(gaps) - gaps[0]
