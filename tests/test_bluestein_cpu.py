"""The shortest exact Bluestein length used by the ring-FFT plan.

Bluestein writes a length-n DFT as a cyclic convolution with the chirp
b_t = exp(i pi t^2 / n) at offsets -(n-1) .. n-1.  The chirp is even in t, so
at a cyclic length L = 2n - 2 the only two offsets that share an index,
+(n-1) and -(n-1), need the same value there, and the convolution is exact;
at L = 2n - 3 offsets with different chirp values collide.  These tests check
that reading with numpy FFTs alone (no library code): the plan picks the
shortest 5-smooth L >= 2n - 2.
"""
import numpy as np
import pytest


def bluestein_dft(x, L):
    n = x.size
    t = np.arange(n)
    b = np.exp(1j * np.pi * ((t * t) % (2 * n)) / n)  # exact angle reduction
    ext = np.zeros(L, dtype=complex)
    ext[:n] = b
    ext[L - t[1:]] = b[1:]  # the chirp at negative offsets, t -> L - t
    a = np.zeros(L, dtype=complex)
    a[:n] = x * np.conj(b)
    y = np.fft.ifft(np.fft.fft(a) * np.fft.fft(ext))
    return np.conj(b) * y[:n]


@pytest.mark.parametrize("n", [3, 5, 7, 11, 139, 641, 683, 2049])
def test_bluestein_exact_at_2n_minus_2(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.fft.fft(x)
    got = bluestein_dft(x, 2 * n - 2)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("n", [5, 11, 139, 2049])
def test_bluestein_one_point_shorter_is_wrong(n):
    """At 2n - 3 the offsets n-1 and -(n-2) (and n-2 and -(n-1)) collide and
    the outputs next to k = n - 1 take a wrong chirp value.  Near t = n the
    chirp's phase turns by almost 2 pi per step, so the two values differ by
    about 3 pi / n: an error of a few 1e-4 of the rms output at n = 2049,
    against rounding (1e-15) at 2n - 2."""
    rng = np.random.default_rng(n + 1)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.fft.fft(x)
    scale = np.sqrt(np.mean(np.abs(ref) ** 2))
    bad = np.abs(bluestein_dft(x, 2 * n - 3) - ref) / scale
    good = np.abs(bluestein_dft(x, 2 * n - 2) - ref) / scale
    assert bad.max() > 1e-5 and good.max() < 1e-12
    assert set(np.flatnonzero(bad > 1e-9)) <= {0, 1, n - 2, n - 1}
