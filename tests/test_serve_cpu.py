"""Host-side checks of the serving layer that need no GPU: the admission policy
(first come first served under a slot count and an HBM budget), the serving
workload recipe, and the host-side argument checks of the plan-residency
entry points."""
import ctypes
import os

import numpy as np
import pytest

import sht_inputs as si

sht = pytest.importorskip("paper_1106_0159_amd")
serve = pytest.importorskip("paper_1106_0159_amd.serve")


def test_admission_respects_slots_and_budget():
    a = serve.Admission(budget=100, slots=2)
    s0 = a.try_admit(60)
    assert s0 is not None and a.used == 60
    assert a.try_admit(50) is None  # 110 > 100: must wait
    s1 = a.try_admit(40)
    assert s1 is not None and s1 != s0 and a.used == 100
    assert a.try_admit(0) is None  # no slot left
    a.release(s0, 60)
    assert a.used == 40 and a.try_admit(50) == s0
    assert a.max_used == 100 and a.max_running == 2
    assert a.fits_ever(100) and not a.fits_ever(101)


def test_admission_rejects_bad_configuration():
    with pytest.raises(ValueError):
        serve.Admission(0, 1)
    with pytest.raises(ValueError):
        serve.Admission(10, 0)


def test_admission_random_schedule_never_exceeds_budget():
    """A random arrive/finish schedule: bytes in flight stay within the
    budget, slots are never shared, and the queue is served in order."""
    rng = np.random.default_rng(7)
    budget, slots = 1000, 3
    a = serve.Admission(budget, slots)
    queue = list(rng.integers(1, 700, 300))
    running, admitted = {}, []
    i = 0
    while i < len(queue) or running:
        if running and (i >= len(queue) or rng.random() < 0.4):
            slot = list(running)[rng.integers(len(running))]
            a.release(slot, running.pop(slot))
        while i < len(queue):
            s = a.try_admit(int(queue[i]))
            if s is None:
                break
            assert s not in running
            running[s] = int(queue[i])
            admitted.append(i)
            i += 1
        assert a.used == sum(running.values()) <= budget
        assert len(running) <= slots
    assert admitted == list(range(len(queue)))
    assert a.used == 0 and sorted(a.free) == list(range(slots))


def test_serving_trace_recipe():
    lm, kinds, t = si.serving_trace(4000, 5)
    assert lm.dtype == np.int64 and np.all(lm % 2 == 0)
    assert lm.min() >= 64 and lm.max() <= 4096
    # log-uniform: the median near the geometric mean sqrt(64 * 4096) = 512
    assert 420 <= np.median(lm) <= 620
    assert set(kinds) == {"alm2map", "map2alm"} and 0.45 < np.mean(kinds == "alm2map") < 0.55
    assert t[0] == 0 and np.all(np.diff(t) >= 0)
    assert abs(t[-1] / (len(t) - 1) - 1.0) < 0.1  # unit rate
    lm2, k2, t2 = si.serving_trace(4000, 5)
    assert np.array_equal(lm, lm2) and np.array_equal(k2, kinds) and np.array_equal(t, t2)


def test_request_kind_checked():
    with pytest.raises(ValueError):
        serve.request_bytes("map2map", 8, 8, sht.GeomHandle(si.healpix(4)), 1)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sht.LIB_PATH):
        pytest.skip("libsht.so not built")
    return sht.lib()


def test_request_bytes_counts_input_output_and_workspace(L):
    g = sht.GeomHandle(si.healpix(8))
    for kind in serve.KINDS:
        need, ws = serve.request_bytes(kind, 16, 16, g, 3)
        assert ws == sht.workspace_bytes(16, 16, g, 3)
        assert need == ws + 3 * (g.npix * 8 + sht.nalm(16, 16) * 16)


def test_plan_entry_points_reject_bad_arguments(L):
    g = sht.GeomHandle(si.healpix(2))
    assert L.sht_plan_cache_limits(0, 4) == sht.SHT_EINVAL
    assert L.sht_plan_cache_limits(4, 0) == sht.SHT_EINVAL
    assert L.sht_plan_cache_limits(8, 32) == sht.SHT_OK  # the defaults; empty caches need no device
    assert L.sht_prepare(-1, 0, g.ref(), 0, None) == sht.SHT_EINVAL
    assert L.sht_prepare(4, 5, g.ref(), 0, None) == sht.SHT_EINVAL
    assert L.sht_prepare(4, 4, None, 0, None) == sht.SHT_EINVAL
    assert L.sht_prepare(4, 4, g.ref(), 8, None) == sht.SHT_EUNSUPPORTED  # (4 is SHT_PIN)
    assert L.sht_plan_cache_bytes() == 0  # nothing built in this process


def test_autotune_table_lookup():
    """The tile table's buckets and admissible candidates (no GPU): wave
    tiles of analysis must hold every ring slot of one m."""
    from paper_1106_0159_amd import autotune, ring_slots
    assert autotune.bucket(100, 51) == "l128_s64"
    assert autotune.bucket(5000, 9000) == "l4096_s4096"
    assert autotune.candidates("alm2map", 1000) == [1, 2, 4]
    assert autotune.candidates("map2alm", 100) == [2, 4, 17, 18, 20]
    assert autotune.candidates("map2alm", 300) == [17, 18, 20]
    table = {"alm2map": {"l128_s64": 2}, "map2alm": {"l128_s64": 4, "l512_s512": 4}}
    assert autotune.choose(table, "alm2map", 100, 51) == 2
    assert autotune.choose(table, "map2alm", 100, 51) == 4
    assert autotune.choose(table, "map2alm", 400, 300) == 0  # a wave of 256 slots cannot hold 300
    assert autotune.choose({}, "map2alm", 100, 51) == 0
    assert ring_slots(si.gauss_legendre(129, 257).theta) == 65
    assert ring_slots(si.healpix(16).theta) == 32
