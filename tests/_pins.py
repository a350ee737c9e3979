"""Independent mathematical references used to pin the oracle.

Nothing here calls the oracle or the GPU library.  The references are:
  * closed forms of the normalised associated Legendre functions for l <= 3
    (with the Condon-Shortley phase),
  * the terminating Gauss hypergeometric representation of the Ferrers
    function, evaluated in mpmath with adaptive precision:
      P_l^m(cos t) = (-1)^m (l+m)! / (2^m m! (l-m)!) sin^m t
                     * 2F1(m-l, l+m+1; m+1; sin^2(t/2)),
    normalised by sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),
  * scipy.special.sph_legendre_p / sph_harm_y (library routines).
"""
from __future__ import annotations

import math
from fractions import Fraction

import mpmath
import numpy as np

PI = math.pi


def lam_closed(l: int, m: int, theta: float) -> float:
    """lambda_lm(cos theta) for l <= 3 from the textbook closed forms."""
    x, s = math.cos(theta), math.sin(theta)
    table = {
        (0, 0): 1.0 / math.sqrt(4 * PI),
        (1, 0): math.sqrt(3 / (4 * PI)) * x,
        (1, 1): -math.sqrt(3 / (8 * PI)) * s,
        (2, 0): math.sqrt(5 / (4 * PI)) * (3 * x * x - 1) / 2,
        (2, 1): -math.sqrt(15 / (8 * PI)) * x * s,
        (2, 2): math.sqrt(15 / (32 * PI)) * s * s,
        (3, 0): math.sqrt(7 / (4 * PI)) * (5 * x ** 3 - 3 * x) / 2,
        (3, 1): -math.sqrt(21 / (64 * PI)) * s * (5 * x * x - 1),
        (3, 2): math.sqrt(105 / (32 * PI)) * x * s * s,
        (3, 3): -math.sqrt(35 / (64 * PI)) * s ** 3,
    }
    return table[(l, m)]


def lam_hyper(l: int, m: int, theta: float):
    """lambda_lm(cos theta) as an mpmath number (unbounded exponent range)."""
    dps = 60
    while True:
        with mpmath.workdps(dps):
            th = mpmath.mpf(theta)
            t = mpmath.sin(th / 2) ** 2
            term = mpmath.mpf(1)
            tot = mpmath.mpf(1)
            big = mpmath.mpf(1)
            a, b, c = m - l, l + m + 1, m + 1
            for k in range(l - m):
                term = term * (a + k) * (b + k) / ((c + k) * (k + 1)) * t
                tot += term
                if abs(term) > big:
                    big = abs(term)
            lost = 0 if tot == 0 else int(mpmath.log10(big / abs(tot))) + 1
            if lost + 30 <= dps:
                nrm = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l + m)
                                  / mpmath.factorial(l - m)) / (mpmath.mpf(2) ** m
                                                                * mpmath.factorial(m))
                return (-1) ** m * nrm * mpmath.sin(th) ** m * tot
            dps = lost + 60


def consistent_theta(target: float, tol: float = 1e-19) -> float:
    """A double near ``target`` whose rounded cos and sin satisfy x^2+s^2=1 to ``tol``.

    The Legendre functions of a rounded (x, s) pair only obey identities such
    as the addition theorem up to |x^2 + s^2 - 1| / s^2; picking a colatitude
    where the pair is consistent makes those identities sharp pins.
    """
    best, best_d = target, 1.0
    th = target
    for _ in range(200000):
        x, s = math.cos(th), math.sin(th)
        d = abs(Fraction(x) ** 2 + Fraction(s) ** 2 - 1)
        if d < best_d:
            best, best_d = th, d
            if d < tol:
                return th
        th = math.nextafter(th, 4.0)
    return best
