"""Oracle results that several GPU tests compare against, computed once per
test session (the full-size ones take tens of seconds of host time)."""
import functools

import numpy as np

import oracle
import sht_inputs as si


@functools.lru_cache(maxsize=None)
def config2():
    """HEALPix N_side = 1024, lmax = mmax = 2048, power-law a_lm of the
    configuration-2 seed (map 0 of the batched runs too)."""
    return si.healpix(1024), 2048, si.powerlaw_alm(2048, 2048, si.config_seed(2))


@functools.lru_cache(maxsize=None)
def config2_map():
    """The oracle's alm2map of config2() over every ring (read only)."""
    g, lmax, a = config2()
    m = oracle.alm2map(lmax, lmax, g, a)
    m.setflags(write=False)
    return m


@functools.lru_cache(maxsize=None)
def config2_analysis_input():
    """The map that the config-2 analysis tests feed in: white noise (scale
    1e-2) plus the oracle's synthesis of the power-law a_lm, and the oracle's
    map2alm of it over every m."""
    g, lmax, _ = config2()
    s = si.random_map(g, 77) * 1e-2 + config2_map()
    ref = oracle.map2alm(lmax, lmax, g, s)
    s.setflags(write=False)
    ref.setflags(write=False)
    return s, ref


def relrms(got, ref):
    den = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / (den if den > 0 else 1.0)
