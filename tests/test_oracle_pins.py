"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: textbook
closed forms, an independent hypergeometric representation in multiple
precision, library routines (scipy, numpy.fft), identities (addition
theorem, adjointness, Gauss-Legendre exactness) and brute-force double sums.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import sph_harm_y, sph_legendre_p

import oracle
import sht_inputs as si
from _pins import consistent_theta, lam_closed, lam_hyper

RNG = np.random.default_rng(20240611)


# ------------------------------------------------------------------ P1
@pytest.mark.parametrize("theta", [0.0, 1e-3, 0.4, 1.0, math.pi / 2, 2.2, 3.1, math.pi])
def test_closed_forms_l_le_3(theta):
    for m in range(4):
        v = oracle.plm(3, m, theta)
        for l in range(m, 4):
            ref = lam_closed(l, m, theta)
            assert abs(v[l - m] - ref) <= 2e-15 * max(1.0, abs(ref)), (l, m, theta)


def test_scipy_sph_legendre_p_moderate_l():
    lmax = 500
    for theta in [0.05, 0.7, 1.5707, 2.9]:
        for m in [0, 1, 2, 17, 100, 250, 499, 500]:
            v = oracle.plm(lmax, m, theta)
            ls = np.arange(m, lmax + 1)
            ref = sph_legendre_p(ls, m, theta)
            env = np.sqrt((2 * ls + 1) / (4 * math.pi))
            assert np.all(np.abs(v - ref) <= 1e-12 * env), (theta, m)


# ------------------------------------------------------------------ P2
@pytest.mark.parametrize("target", [0.01, 0.05, 0.3, 1.2])
def test_addition_theorem(target):
    theta = consistent_theta(target)
    lmax = 2048
    tot = np.zeros(lmax + 1)
    for m in range(lmax + 1):
        p = oracle.plm(lmax, m, theta)
        tot[m:] += (1.0 if m == 0 else 2.0) * p * p
    ls = np.arange(lmax + 1)
    rel = np.abs(tot / ((2 * ls + 1) / (4 * math.pi)) - 1.0)
    # forward error of the double recurrence near the pole: ~4e-13 by l=360, ~5e-13 at l=1800
    assert np.all(rel <= np.minimum(2e-15 * ls, 1e-12) + 1e-14), (theta, rel.max(), int(rel.argmax()))


def test_poles():
    lmax = 300
    for theta, sgn in [(0.0, 1.0), (math.pi, -1.0)]:
        for m in range(0, 6):
            v = oracle.plm(lmax, m, theta)
            ls = np.arange(m, lmax + 1)
            if m == 0:
                ref = sgn ** ls * np.sqrt((2 * ls + 1) / (4 * math.pi))
                assert np.allclose(v, ref, rtol=1e-13, atol=0)
            else:  # sin(pi) is 1.2e-16 in double, so P_lm(-1) is tiny but not 0
                assert np.all(np.abs(v) <= 1e-12), (theta, m)


# ------------------------------------------------------------------ P3
HEALPIX_1024_FIRST = 2.0 * math.asin(1.0 / (math.sqrt(6.0) * 1024))


@pytest.mark.parametrize("l,m,theta", [
    (2048, 2048, HEALPIX_1024_FIRST),    # ~1e-6346: many rescalings in the seed
    (2048, 1500, HEALPIX_1024_FIRST),
    (2048, 2, HEALPIX_1024_FIRST),
    (4096, 4096, 1e-3),                  # ~1e-12288
    (4096, 100, 1e-3),
    (4096, 30, 2e-3),
    (2048, 1000, 0.3),                   # grows from 1e-137 through the turning point
    (2048, 1000, 0.8),
    (1200, 700, 2.6),
])
def test_extended_range_against_hypergeometric(l, m, theta):
    mant, e = oracle.plm_ext(l, m, theta)
    ref = lam_hyper(l, m, theta)
    got = mpmath.mpf(float(mant[-1])) * mpmath.mpf(2) ** int(e[-1])
    assert ref != 0
    assert abs(got / ref - 1) < 1e-10, (l, m, theta, mpmath.nstr(got, 12), mpmath.nstr(ref, 12))


def test_extended_range_whole_column_matches_hypergeometric():
    """Every l of one deep column, including the region where rescaling switches."""
    theta, m, lmax = 0.02, 600, 1400
    mant, e = oracle.plm_ext(lmax, m, theta)
    for l in range(m, lmax + 1, 40):
        ref = lam_hyper(l, m, theta)
        got = mpmath.mpf(float(mant[l - m])) * mpmath.mpf(2) ** int(e[l - m])
        assert abs(got / ref - 1) < 1e-10, l


# ------------------------------------------------------------------ P4
def _ring_phis(g, r):
    return g.phi0[r] + 2 * math.pi * np.arange(g.nphi[r]) / g.nphi[r]


@pytest.mark.parametrize("l,m,coef", [(5, 3, 1.0), (9, 9, 1.0), (9, 7, 1j), (12, 0, 1.0), (14, 11, 0.3 - 0.7j)])
def test_single_mode_maps_with_aliasing(l, m, coef):
    # rings with nphi < 2m+1 alias the mode; the plain definition handles it
    theta = np.array([0.3, 1.1, 1.9, 2.8])
    nphi = np.array([3, 8, 23, 5], dtype=np.int32)
    phi0 = np.array([0.0, 0.25, 1.3, -0.7])
    g = si._pack(theta, nphi, phi0, np.ones(4), "single")
    lmax = 16
    a = np.zeros(si.nalm(lmax, lmax), dtype=np.complex128)
    a[si.alm_index(l, m, lmax)] = coef
    mp = oracle.alm2map(lmax, lmax, g, a)
    for r in range(4):
        lam = sph_legendre_p(l, m, theta[r])
        phis = _ring_phis(g, r)
        if m == 0:
            ref = np.full(nphi[r], coef.real * lam)
        else:
            ref = 2 * np.real(coef * np.exp(1j * m * phis)) * lam
        got = mp[g.ofs[r]: g.ofs[r] + nphi[r]]
        assert np.allclose(got, ref, rtol=0, atol=1e-14), (r, got, ref)


# ------------------------------------------------------------------ brute force
def _random_geometry(nr, seed):
    rng = np.random.default_rng(seed)
    theta = np.sort(rng.uniform(0.05, math.pi - 0.05, nr))
    nphi = rng.integers(1, 30, nr).astype(np.int32)
    phi0 = rng.uniform(-1, 7, nr)
    w = rng.uniform(0.1, 1.0, nr)
    return si._pack(theta, nphi, phi0, w, "random")


def _brute_map(lmax, mmax, g, a):
    out = np.zeros(g.npix)
    for r in range(g.nrings):
        phis = _ring_phis(g, r)
        acc = np.zeros(g.nphi[r], dtype=np.complex128)
        for l in range(lmax + 1):
            for m in range(-min(l, mmax), min(l, mmax) + 1):
                alm = a[si.alm_index(l, abs(m), lmax)]
                if m < 0:
                    alm = (-1) ** m * np.conj(alm)
                elif m == 0:
                    alm = alm.real
                acc += alm * sph_harm_y(l, m, g.theta[r], phis)
        out[g.ofs[r]: g.ofs[r] + g.nphi[r]] = acc.real
    return out


@pytest.mark.parametrize("lmax,mmax", [(0, 0), (1, 1), (6, 6), (7, 4)])
def test_alm2map_brute_force(lmax, mmax):
    g = _random_geometry(9, 3 + lmax)
    a = si.uniform_alm(lmax, mmax, 5 + lmax)
    a[: lmax + 1] += 0.37j  # Im a_l0 must be ignored
    got = oracle.alm2map(lmax, mmax, g, a)
    ref = _brute_map(lmax, mmax, g, a)
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("lmax,mmax", [(0, 0), (2, 2), (6, 6), (7, 3)])
def test_map2alm_brute_force(lmax, mmax):
    g = _random_geometry(8, 11 + lmax)
    s = si.random_map(g, 13 + lmax)
    got = oracle.map2alm(lmax, mmax, g, s)
    ref = np.zeros_like(got)
    for m in range(mmax + 1):
        for l in range(m, lmax + 1):
            acc = 0j
            for r in range(g.nrings):
                phis = _ring_phis(g, r)
                y = sph_harm_y(l, m, g.theta[r], phis)
                acc += np.sum(g.weight[r] * s[g.ofs[r]: g.ofs[r] + g.nphi[r]] * np.conj(y))
            ref[si.alm_index(l, m, lmax)] = acc
    ref[: lmax + 1] = ref[: lmax + 1].real
    assert np.max(np.abs(got - ref)) < 1e-13
    assert np.all(got[: lmax + 1].imag == 0.0)


# ------------------------------------------------------------------ azimuthal stage vs numpy.fft
def test_delta2map_matches_numpy_fft():
    mmax = 40
    nphi = np.array([7, 81, 100, 13, 64], dtype=np.int32)  # some < 2 mmax + 1 (aliasing)
    phi0 = np.array([0.0, 0.3, -1.1, 2.0, 0.5])
    g = si._pack(np.linspace(0.3, 2.8, 5), nphi, phi0, np.ones(5), "fft")
    d = RNG.standard_normal((5, mmax + 1)) + 1j * RNG.standard_normal((5, mmax + 1))
    got = oracle.delta2map(mmax, g, d)
    for r in range(5):
        n = int(nphi[r])
        ms = np.arange(mmax + 1)
        c = d[r] * np.exp(1j * ms * phi0[r]) * np.where(ms == 0, 1.0, 2.0)
        c[0] = d[r, 0].real
        folded = np.zeros(n, dtype=np.complex128)
        np.add.at(folded, ms % n, c)
        ref = np.real(np.fft.ifft(folded) * n)
        assert np.allclose(got[g.ofs[r]: g.ofs[r] + n], ref, rtol=0, atol=1e-12)


def test_map2delta_matches_numpy_fft():
    mmax = 40
    nphi = np.array([5, 81, 100, 17], dtype=np.int32)
    phi0 = np.array([0.1, -0.3, 1.1, 4.0])
    w = np.array([0.5, 2.0, 1.0, 0.25])
    g = si._pack(np.linspace(0.3, 2.8, 4), nphi, phi0, w, "fft")
    s = si.random_map(g, 99)
    got = oracle.map2delta(mmax, g, s)
    for r in range(4):
        n = int(nphi[r])
        f = np.fft.fft(s[g.ofs[r]: g.ofs[r] + n])
        ms = np.arange(mmax + 1)
        ref = w[r] * f[ms % n] * np.exp(-1j * ms * phi0[r])
        assert np.allclose(got[r], ref, rtol=0, atol=1e-12)


def test_map2alm_subset_of_m_matches_full():
    g = si.healpix(4)
    lmax = 10
    s = si.random_map(g, 3)
    full = oracle.map2alm(lmax, lmax, g, s)
    part = oracle.map2alm(lmax, lmax, g, s, ms=[7, 2])
    for m in (2, 7):
        i0, i1 = si.alm_index(m, m, lmax), si.alm_index(lmax, m, lmax) + 1
        assert np.array_equal(part[i0:i1], full[i0:i1])


def test_alm2map_subset_of_rings_matches_full():
    g = si.healpix(4)
    lmax = 8
    a = si.powerlaw_alm(lmax, lmax, 1)
    full = oracle.alm2map(lmax, lmax, g, a)
    rings = [14, 0, 6]
    part = oracle.alm2map(lmax, lmax, g, a, rings=rings)
    for r in rings:
        sl = slice(g.ofs[r], g.ofs[r] + g.nphi[r])
        assert np.array_equal(part[sl], full[sl])


# ------------------------------------------------------------------ P5
@pytest.mark.parametrize("lmax,mmax", [(1, 1), (16, 16), (64, 64), (63, 20)])
def test_gauss_legendre_round_trip(lmax, mmax):
    g = si.gauss_legendre(lmax + 1, 2 * mmax + 1)
    for a in (si.powerlaw_alm(lmax, mmax, 7), si.uniform_alm(lmax, mmax, 8)):
        a = a.copy()
        if lmax >= 1:
            a[1] = 0.5  # non-zero dipole so power-law maps are not trivial at l=1
        back = oracle.map2alm(lmax, mmax, g, oracle.alm2map(lmax, mmax, g, a))
        err = np.linalg.norm(back - a) / np.linalg.norm(a)
        assert err < 2e-14, err


@pytest.mark.slow
def test_gauss_legendre_round_trip_lmax_256():
    lmax = 256
    g = si.gauss_legendre(lmax + 1, 2 * lmax + 1)
    a = si.uniform_alm(lmax, lmax, 9)
    back = oracle.map2alm(lmax, lmax, g, oracle.alm2map(lmax, lmax, g, a))
    assert np.linalg.norm(back - a) / np.linalg.norm(a) < 5e-14


# ------------------------------------------------------------------ P6
def _alm_dot(a, b, lmax):
    m0 = slice(0, lmax + 1)
    return float(np.sum(a[m0].real * b[m0].real) + 2 * np.sum((np.conj(a[lmax + 1:]) * b[lmax + 1:]).real))


@pytest.mark.parametrize("nside,lmax", [(4, 8), (8, 24), (16, 32)])
def test_adjointness_on_healpix(nside, lmax):
    g = si.healpix(nside)
    a = si.uniform_alm(lmax, lmax, 17)
    s = si.random_map(g, 18)
    lhs = _alm_dot(a, oracle.map2alm(lmax, lmax, g, s), lmax)
    w = np.repeat(g.weight, g.nphi)
    rhs = float(np.sum(w * s * oracle.alm2map(lmax, lmax, g, a)))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.sqrt(np.sum(w * s * s)))


# ------------------------------------------------------------------ Im a_l0 handling
def test_imag_part_of_m0_ignored_and_zeroed():
    g = si.healpix(4)
    lmax = 8
    a = si.uniform_alm(lmax, lmax, 21)
    b = a.copy()
    b[: lmax + 1] += 1j * np.linspace(1, 2, lmax + 1)
    assert np.array_equal(oracle.alm2map(lmax, lmax, g, a), oracle.alm2map(lmax, lmax, g, b))
    out = oracle.map2alm(lmax, lmax, g, si.random_map(g, 2))
    assert np.all(out[: lmax + 1].imag == 0.0)


def test_delta_m0_is_real():
    g = si.healpix(2)
    lmax = 6
    a = si.uniform_alm(lmax, lmax, 4)
    a[: lmax + 1] += 0.5j
    d = oracle.delta_syn(lmax, lmax, g, a)
    assert np.all(d[:, 0].imag == 0.0)
    # and Delta_0 is the real l-sum of a_l0 lambda_l0
    for r in range(g.nrings):
        ref = sum(a[l].real * sph_legendre_p(l, 0, g.theta[r]) for l in range(lmax + 1))
        assert abs(d[r, 0].real - ref) < 1e-14


def test_invalid_arguments_rejected():
    g = si.healpix(2)
    with pytest.raises(ValueError):
        oracle.plm(3, 4, 0.5)
    with pytest.raises(ValueError):
        oracle.plm(3, 1, -0.1)
    with pytest.raises(ValueError):
        oracle.alm2map(4, 5, g, np.zeros(40, dtype=np.complex128))
