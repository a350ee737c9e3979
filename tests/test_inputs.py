"""Seeded input generators: geometry invariants and a_lm statistics (no GPU)."""
import math

import numpy as np
import pytest

import sht_inputs as si


@pytest.mark.parametrize("nside", [1, 2, 4, 64, 1024])
def test_healpix_geometry(nside):
    g = si.healpix(nside)
    assert g.nrings == 4 * nside - 1
    assert int(g.nphi.sum()) == 12 * nside * nside == g.npix
    assert abs(float(np.sum(g.weight * g.nphi)) - 4 * math.pi) < 1e-12
    assert np.all(np.diff(g.theta) > 0)
    # mirror symmetry of the ring set
    assert np.allclose(g.theta + g.theta[::-1], math.pi, rtol=0, atol=1e-15)
    assert np.array_equal(g.nphi, g.nphi[::-1])
    # equatorial belt
    assert np.all(g.nphi[nside - 1: 3 * nside] == 4 * nside)
    # ring z-values from the published ring scheme
    i = np.arange(1, nside)
    if nside > 1:
        assert np.allclose(np.cos(g.theta[: nside - 1]), 1 - i * i / (3.0 * nside * nside), rtol=0, atol=1e-15)
    ib = np.arange(nside, 3 * nside + 1)
    assert np.allclose(np.cos(g.theta[nside - 1: 3 * nside]), (4 * nside - 2 * ib) / (3.0 * nside), atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 5, 64, 257, 1025])
def test_gauss_legendre_geometry(n):
    g = si.gauss_legendre(n, 2 * n + 1)
    x = np.cos(g.theta)
    w = g.weight * g.nphi / (2 * math.pi)
    assert abs(w.sum() - 2) < 1e-14
    # exact for polynomials of degree <= 2n-1
    for k in range(0, n):
        assert abs(np.sum(w * x ** (2 * k)) * (2 * k + 1) / 2 - 1) < 2e-14
    assert np.all(np.diff(g.theta) > 0)
    from numpy.polynomial import legendre as L
    xr, _ = L.leggauss(n)
    assert np.allclose(np.sort(x), xr, rtol=0, atol=1e-15)


def test_powerlaw_alm_statistics():
    lmax = 512
    a = si.powerlaw_alm(lmax, lmax, si.config_seed(2))
    assert a.shape == (si.nalm(lmax, lmax),)
    assert np.all(a[: lmax + 1].imag == 0)
    assert a[0] == 0 and a[1] == 0
    # empirical C_l ~ 1/(l(l+1))
    for l in (50, 200, 500):
        idx = [si.alm_index(l, m, lmax) for m in range(l + 1)]
        v = a[idx]
        cl = (abs(v[0]) ** 2 + 2 * np.sum(np.abs(v[1:]) ** 2)) / (2 * l + 1)
        assert 0.7 < cl * l * (l + 1) < 1.3
    b = si.powerlaw_alm(lmax, lmax, si.config_seed(2))
    assert np.array_equal(a, b)  # seeded


def test_alm_index_layout():
    lmax, mmax = 9, 5
    seen = []
    for m in range(mmax + 1):
        for l in range(m, lmax + 1):
            seen.append(si.alm_index(l, m, lmax))
    assert seen == list(range(si.nalm(lmax, mmax)))
