"""Continuous-batching server for alm2map / map2alm requests of mixed size.

Requests of any (lmax, geometry) arrive over time.  Each is admitted as soon
as a slot (one HIP stream) and its share of an HBM budget are free.  The work
of admitted requests therefore overlaps on the device, and newcomers join while
others run.  A request is retired once its completion event has fired.

The budget charges each request what the paper's memory model (Sec. 4.1.2)
counts per transform: its input, its output and the Delta workspace of the
library call.  The plan tables of every grid stay resident beside it
(`prepare`, built once per grid and charged once, `sht_plan_cache_bytes`).

Every step of a transform runs in the HIP library through the binding; this
module only schedules requests and keeps their timestamps.  Results do not
depend on the mix: each request runs alone on its own stream, and the kernels
are deterministic, so a result is bitwise the same alone and among others.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import (GeomHandle, SHT_EINVAL, ShtError, alm2map, map2alm, nalm, plan_cache_bytes,
               plan_cache_limits, prepare, workspace_bytes)

KINDS = ("alm2map", "map2alm")


@dataclasses.dataclass
class Request:
    """One transform.  `data` is the device input: complex128 a_lm
    [nmaps, nalm] (alm2map) or float64 maps [nmaps, npix] (map2alm)."""
    kind: str
    lmax: int
    geom: GeomHandle
    data: object
    mmax: int | None = None
    arrival: float | None = None  # host perf_counter() seconds; set by submit() if None
    rid: int = -1
    # set by the server
    status: str = "new"  # new -> pending -> running -> done | rejected | failed
    error: str = ""
    need: int = 0
    ws_bytes: int = 0
    result: object = None
    t_admit: float = 0.0
    t_done: float = 0.0
    ready: object = None  # event on the submitting stream: the input is complete there

    def __post_init__(self):
        if self.kind not in KINDS:
            raise ValueError(f"unknown request kind {self.kind!r}")
        if self.mmax is None:
            self.mmax = self.lmax

    @property
    def nmaps(self) -> int:
        per = nalm(self.lmax, self.mmax) if self.kind == "alm2map" else self.geom.npix
        return max(1, self.data.numel() // per)

    @property
    def latency(self) -> float:
        """Arrival to completion, seconds (the completion event is placed on
        the host clock to within the few tens of microseconds of one
        synchronisation)."""
        return self.t_done - self.arrival


def request_bytes(kind: str, lmax: int, mmax: int, geom: GeomHandle, nmaps: int, flags: int = 0):
    """(bytes one request holds while it runs: input + output + workspace,
    workspace bytes)."""
    if kind not in KINDS:
        raise ValueError(f"unknown request kind {kind!r}")
    ws = workspace_bytes(lmax, mmax, geom, nmaps, flags)
    if ws == 0:
        raise ShtError(SHT_EINVAL, "sht_workspace_bytes")
    return ws + nmaps * (geom.npix * 8 + nalm(lmax, mmax) * 16), ws


class Admission:
    """First-come first-served admission under a slot count and a byte budget.

    The head of the queue is admitted when a slot is free and its bytes fit
    beside those in flight; a later request never overtakes it, so the order of
    admission is the order of arrival.  A request larger than the whole budget
    can never run and is rejected at submission."""

    def __init__(self, budget: int, slots: int):
        if budget <= 0 or slots <= 0:
            raise ValueError("budget and slots must be positive")
        self.budget = int(budget)
        self.free = list(range(slots - 1, -1, -1))
        self.used = 0
        self.max_used = 0
        self.max_running = 0
        self.nslots = slots

    def fits_ever(self, need: int) -> bool:
        return need <= self.budget

    def try_admit(self, need: int):
        """Slot index for a request of `need` bytes, or None if it must wait."""
        if not self.free or self.used + need > self.budget:
            return None
        self.used += need
        self.max_used = max(self.max_used, self.used)
        slot = self.free.pop()
        self.max_running = max(self.max_running, self.nslots - len(self.free))
        return slot

    def release(self, slot: int, need: int) -> None:
        self.used -= need
        self.free.append(slot)


class Server:
    """Schedules requests over `slots` HIP streams (default priority) within
    `hbm_budget` bytes.  `flags` is the precision mode of every request
    (0 = FP64, SHT_MIXED = FP32 matrix-core contraction)."""

    def __init__(self, hbm_budget: int = 64 << 30, slots: int = 4, flags: int = 0, keep_results: bool = True):
        import torch
        self.torch = torch
        self.flags = flags
        self.keep_results = keep_results
        self.adm = Admission(hbm_budget, slots)
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.pending = collections.deque()
        self.running = {}  # slot -> (request, completion event, workspace)
        self.finished = []
        self._next_id = 0
        # host time of a reference event: completion events are placed on the
        # host clock through their device-side distance to it
        self._ref = torch.cuda.Event(enable_timing=True)
        self._ref.record()
        self._ref.synchronize()
        self._t_ref = time.perf_counter()

    # -- plans
    def prepare(self, geom: GeomHandle, lmax: int, mmax: int | None = None) -> None:
        prepare(geom, lmax, mmax, flags=self.flags)

    @staticmethod
    def reserve_plans(n_grids: int) -> None:
        """Let the plan cache keep `n_grids` grids (and their coefficient
        tables) resident."""
        plan_cache_limits(max(8, n_grids), max(32, n_grids))

    @staticmethod
    def plan_bytes() -> int:
        return plan_cache_bytes()

    # -- requests
    def submit(self, req: Request) -> bool:
        """Queue a request; False (status 'rejected') if it can never fit.

        The input may still be in production on the caller's current stream:
        an event recorded there now orders the request's own stream after it
        (the request's transform waits for it on the device, not the host)."""
        if req.arrival is None:
            req.arrival = time.perf_counter()
        req.ready = self.torch.cuda.Event()
        req.ready.record(self.torch.cuda.current_stream(req.data.device))
        req.rid = self._next_id
        self._next_id += 1
        req.need, req.ws_bytes = request_bytes(req.kind, req.lmax, req.mmax, req.geom, req.nmaps, self.flags)
        if not self.adm.fits_ever(req.need):
            req.status = "rejected"
            self.finished.append(req)
            return False
        req.status = "pending"
        self.pending.append(req)
        return True

    def _launch(self, slot: int, req: Request) -> None:
        torch = self.torch
        s = self.streams[slot]
        ev = torch.cuda.Event(enable_timing=True)
        req.t_admit = time.perf_counter()
        try:
            with torch.cuda.stream(s):
                # the slot stream runs after the input's producer, and the
                # input's memory is not reused while this stream may read it
                s.wait_event(req.ready)
                req.data.record_stream(s)
                ws = torch.empty(req.ws_bytes, dtype=torch.uint8, device=req.data.device)
                f = alm2map if req.kind == "alm2map" else map2alm
                req.result = f(req.data, req.geom, req.lmax, req.mmax, ws=ws, stream=s, flags=self.flags)
                ev.record(s)
        except RuntimeError as e:
            # a library rejection (ShtError: nothing was enqueued) or a failed
            # allocation: the request fails, its slot and bytes go back
            req.status, req.error = "failed", str(e)
            self.adm.release(slot, req.need)
            self.finished.append(req)
            return
        req.status = "running"
        self.running[slot] = (req, ev, ws)

    def poll(self) -> int:
        """Retire completed requests, admit what fits; returns the number of
        requests pending or running."""
        for slot in [k for k, (_, ev, _) in self.running.items() if ev.query()]:
            req, ev, _ = self.running.pop(slot)
            req.t_done = self._t_ref + self._ref.elapsed_time(ev) / 1e3
            req.status = "done"
            if not self.keep_results:
                req.result = None
            self.adm.release(slot, req.need)
            self.finished.append(req)
        while self.pending:
            slot = self.adm.try_admit(self.pending[0].need)
            if slot is None:
                break
            self._launch(slot, self.pending.popleft())
        return len(self.pending) + len(self.running)

    def drain(self, sleep: float = 20e-6) -> None:
        while self.poll():
            time.sleep(sleep)

    def run_trace(self, requests, sleep: float = 20e-6) -> None:
        """Submit `requests` (sorted by `arrival`, seconds from now) as their
        arrival times come, admitting and retiring as the device frees up."""
        t0 = time.perf_counter()
        i, n = 0, len(requests)
        while True:
            now = time.perf_counter() - t0
            while i < n and requests[i].arrival <= now:
                requests[i].arrival += t0
                self.submit(requests[i])
                i += 1
            busy = self.poll()
            if i >= n and busy == 0:
                break
            time.sleep(sleep)

    # -- report
    def stats(self) -> dict:
        done = [r for r in self.finished if r.status == "done"]
        lat = np.array([r.latency for r in done]) * 1e3
        rejected = sum(r.status == "rejected" for r in self.finished)
        failed = sum(r.status == "failed" for r in self.finished)
        if not done:
            return {"done": 0, "rejected": rejected, "failed": failed}
        span = max(r.t_done for r in done) - min(r.arrival for r in done)
        maps = sum(r.nmaps for r in done)
        return {"done": len(done), "rejected": rejected, "failed": failed,
                "maps_per_s": maps / span, "span_s": span,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_ms": float(lat.max()), "max_running": self.adm.max_running,
                "max_used_bytes": self.adm.max_used, "budget_bytes": self.adm.budget}
