"""Continuous-batching request server for RIDC integrations.

Requests (a problem, its initial data, its number of time steps) arrive over time.  The server
keeps every admitted request resident on the device with its level rings, and advances all
resident requests together, a few pipeline steps per tick, through grouped launches
(``ridc_advance``): a request that arrives while others are running joins the running batch at
its own pipeline step 0 at the next tick.  A request is admitted when a slot is free and its
device footprint (``ridc_footprint_bytes``) fits the remaining HBM budget; finished requests are
read out, their memory freed, and their latency (arrival to result) recorded.  Grouping never
changes a request's result: it is bitwise the same alone and in the mix.

The server drives an *executor* (``GpuExecutor`` here; tests substitute a host-side fake with
the same interface):

``footprint(req) -> int``          device bytes the request needs while resident
``start(req) -> slot``             allocate and arm (load u0, zero pipeline steps done)
``advance(slots, k)``              advance every slot by up to k pipeline steps (grouped)
``remaining(slot) -> int``         pipeline steps left
``finish(slot) -> array``          read the top level (raises on a non-finite result)
``release(slot)``                  free the slot's device memory
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    prob: dict
    u0: Any
    nsteps: int
    prec: str = "fp32"
    t_arrival: float = 0.0
    # filled by the server
    t_admit: float | None = None
    t_done: float | None = None
    status: str = "queued"          # queued | running | done | failed | cancelled | rejected
    result: Any = None
    error: str | None = None

    @property
    def unknowns(self) -> int:
        n = int(self.prob["n"])
        return n if self.prob["dim"] == 1 else n * n

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.t_arrival


class GpuExecutor:
    """Executor over the HIP library: one ``Ridc`` handle per resident request."""

    def __init__(self, stream=None):
        from . import ridc
        self._ridc = ridc
        self._stream = stream
        self._slots = {}
        self._next = 0

    def footprint(self, req: Request) -> int:
        return self._ridc.footprint_bytes(req.prob, prec=req.prec)

    def start(self, req: Request) -> int:
        import torch
        s = self._ridc.Ridc(req.prob, prec=req.prec, stream=self._stream)
        u0 = req.u0
        if not isinstance(u0, torch.Tensor):
            u0 = torch.tensor(np.asarray(u0).reshape(-1), dtype=torch.float64, device="cuda")
        s.begin(u0, req.nsteps)
        slot = self._next
        self._next += 1
        self._slots[slot] = (s, u0)
        return slot

    def advance(self, slots, k: int):
        if slots:
            self._ridc.advance([self._slots[i][0] for i in slots], k)

    def remaining(self, slot: int) -> int:
        return self._slots[slot][0].remaining()

    def finish(self, slot: int):
        import torch
        s, u0 = self._slots[slot]
        out = torch.empty(s.npts, dtype=torch.float64, device="cuda")
        s.read(out)
        s.sync()                       # raises RidcError(RIDC_E_NONFINITE) on NaN/Inf
        return out

    def release(self, slot: int):
        s, _ = self._slots.pop(slot)
        s.close()


class Server:
    """Admission by HBM footprint and slots, continuous batching, latency bookkeeping."""

    def __init__(self, executor, hbm_budget: int, max_slots: int = 64, tick_steps: int = 8,
                 clock=time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.tick_steps = int(tick_steps)
        self.clock = clock
        self.queue = collections.deque()
        self.running = {}                  # slot -> (request, bytes)
        self.used = 0
        self.done = []
        self.peak_used = 0
        self.peak_running = 0
        self.ticks = 0

    # -- requests --------------------------------------------------------------------------
    def submit(self, req: Request):
        fp = self.ex.footprint(req)
        if fp <= 0 or fp > self.budget:
            req.status = "rejected"
            req.error = "footprint exceeds the HBM budget" if fp > 0 else "invalid request"
            self.done.append(req)
            return
        req.status = "queued"
        self.queue.append((req, fp))

    def cancel(self, rid: int) -> bool:
        for i, (req, fp) in enumerate(self.queue):
            if req.rid == rid:
                del self.queue[i]
                req.status = "cancelled"
                self.done.append(req)
                return True
        for slot, (req, fp) in list(self.running.items()):
            if req.rid == rid:
                self._retire(slot, "cancelled")
                return True
        return False

    # -- scheduling ------------------------------------------------------------------------
    def _admit(self):
        # first-come first-served; a request that does not fit lets smaller ones behind it in
        # (backfill), so one large request cannot idle the device
        kept = collections.deque()
        while self.queue:
            req, fp = self.queue.popleft()
            if len(self.running) < self.max_slots and self.used + fp <= self.budget:
                try:
                    slot = self.ex.start(req)
                except Exception as e:  # noqa: BLE001 - the request fails, the server goes on
                    req.status = "failed"
                    req.error = str(e)
                    req.t_done = self.clock()
                    self.done.append(req)
                    continue
                req.status = "running"
                req.t_admit = self.clock()
                self.running[slot] = (req, fp)
                self.used += fp
            else:
                kept.append((req, fp))
        self.queue = kept
        self.peak_used = max(self.peak_used, self.used)
        self.peak_running = max(self.peak_running, len(self.running))

    def _retire(self, slot: int, status: str, result=None, error=None):
        req, fp = self.running.pop(slot)
        self.ex.release(slot)
        self.used -= fp
        req.status = status
        req.result = result
        req.error = error
        req.t_done = self.clock()
        self.done.append(req)

    def tick(self):
        """Admit, advance every resident request by up to tick_steps, retire finished ones."""
        self._admit()
        if not self.running:
            return
        slots = list(self.running)
        self.ex.advance(slots, self.tick_steps)
        self.ticks += 1
        for slot in slots:
            if self.ex.remaining(slot) == 0:
                try:
                    out = self.ex.finish(slot)
                except Exception as e:  # noqa: BLE001 - e.g. a non-finite result
                    self._retire(slot, "failed", error=str(e))
                else:
                    self._retire(slot, "done", result=out)

    def idle(self) -> bool:
        return not self.queue and not self.running

    # -- driver ----------------------------------------------------------------------------
    def run(self, arrivals, horizon: float | None = None, max_wall: float | None = None):
        """Serve ``arrivals`` (requests with ``t_arrival`` in seconds from the start, ascending)
        in real time.  Stops admitting new arrivals after ``horizon`` seconds (they are marked
        rejected) and gives up on queued work after ``max_wall`` seconds (marked unserved)."""
        pending = collections.deque(sorted(arrivals, key=lambda r: r.t_arrival))
        t0 = self.clock()
        base = t0
        while pending or not self.idle():
            now = self.clock() - base
            while pending and pending[0].t_arrival <= now:
                req = pending.popleft()
                req.t_arrival = base + req.t_arrival
                if horizon is not None and now > horizon:
                    req.status = "rejected"
                    req.error = "arrived after the serving horizon"
                    self.done.append(req)
                else:
                    self.submit(req)
            if max_wall is not None and now > max_wall:
                for req, _ in self.queue:
                    req.status = "unserved"
                    self.done.append(req)
                self.queue.clear()
                for slot in list(self.running):
                    self._retire(slot, "unserved")
                for req in pending:
                    req.status = "unserved"
                    self.done.append(req)
                pending.clear()
                break
            if self.idle():
                if pending:                      # nothing to do until the next arrival
                    wait = pending[0].t_arrival - (self.clock() - base)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            self.tick()
        return self.stats(self.clock() - t0)

    def stats(self, wall: float) -> dict:
        done = [r for r in self.done if r.status == "done"]
        lat = np.array([r.latency for r in done]) if done else np.array([])
        gps = sum(r.unknowns * r.nsteps for r in done)
        by = collections.Counter(r.status for r in self.done)
        return {
            "completed": len(done),
            "status_counts": dict(by),
            "wall_s": wall,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "completed_grid_point_steps_per_s": gps / wall if wall > 0 else 0.0,
            "completed_requests_per_s": len(done) / wall if wall > 0 else 0.0,
            "peak_hbm_bytes": self.peak_used,
            "peak_resident": self.peak_running,
            "ticks": self.ticks,
        }
