"""Continuous-batching serving loop over resident pools (ia_pool_*).

Events arrive over time (for instance as a Poisson stream).  The loop keeps
one resident pool per size class of events (rows of up to 128, 256, 512 or
1,024 hits by default), each on its own library context (its scratch arena,
a share of the device-memory budget) and its own stream, so the pools'
passes run concurrently on the device.  An arriving event is admitted into
a free row of the smallest class that holds it (a larger class when that one
is full), so the device memory it occupies follows its own size.  The pool's
rows keep their whole search state on the device between passes; every step
runs one helix pass over all rows still searching, so events that arrived at
different times share the launches (continuous batching at the granularity of
a helix pass).  When a step completes, finished rows hand back their helices
and take new events.  An event's latency runs from its arrival to the moment
its result is on the host.

An event's result does not depend on the row, the pool or the other events
(the kernels treat every event independently), which tests/test_gpu_serve.py
checks against ia_find_helices and the oracle.  The device work runs in the
HIP kernels of libia; this module only schedules host-side work.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import Context, Pool, Schedule


@dataclasses.dataclass
class Request:
    rid: int
    hits: np.ndarray            # structured ia_hit records
    arrival: float              # seconds on the loop's clock
    done: float = float("nan")
    helices: np.ndarray = None  # HELIX_DTYPE records
    assigned: np.ndarray = None


DEFAULT_CLASSES = {128: 0.40, 256: 0.35, 512: 0.15, 1024: 0.10}


class _PoolSlot:
    def __init__(self, device, max_hits, budget, sched, max_per_event, rows_cap, torch):
        self.torch = torch
        self.max_hits = max_hits
        self.ctx = Context(device, scratch_bytes=int(budget))
        self.stream = torch.cuda.Stream(device=device)
        rows = min(rows_cap, Pool.capacity(self.ctx, max_hits, sched, max_per_event))
        if rows < 1:
            raise ValueError(f"scratch budget below one {max_hits}-hit row")
        self.pool = Pool(self.ctx, rows, max_hits, sched, max_per_event, stream=self.stream)
        self.rows = rows
        self.occupant = [None] * rows        # Request per occupied row
        self.free = collections.deque(range(rows))
        self.step_ev = None                  # completion event of the step in flight
        self.keep = []                       # device buffers the step in flight reads

    def busy(self):
        return self.step_ev is not None and not self.step_ev.query()


class ServeLoop:
    """Serve requests with resident pools, one per hit-count class.

    classes: {max_hits of a row: share of scratch_budget}."""

    def __init__(self, sched: Schedule, max_per_event=10, scratch_budget=48 << 30, device=0, classes=None,
                 rows_cap=8192):
        import torch
        self.torch = torch
        self.sched = sched
        self.device = device
        classes = dict(DEFAULT_CLASSES if classes is None else classes)
        total = sum(classes.values())
        self.slots = [_PoolSlot(device, int(h), scratch_budget * w / total, sched, max_per_event, rows_cap, torch)
                      for h, w in sorted(classes.items())]
        self.max_out = self.slots[0].pool.max_out
        self.pending = collections.deque()
        self.finished = []

    def capacity(self):
        """{max_hits: rows} of the pools."""
        return {s.max_hits: s.rows for s in self.slots}

    # -- one pool's turn ------------------------------------------------------
    def _collect(self, slot, now_fn):
        done, n_out = slot.pool.poll()
        for r, req in enumerate(slot.occupant):
            if req is None or not done[r]:
                continue
            req.helices, req.assigned = slot.pool.take(r, int(n_out[r]), req.hits.shape[0])
            req.done = now_fn()
            self.finished.append(req)
            slot.occupant[r] = None
            slot.free.append(r)

    def _admit(self, slot):
        torch = self.torch
        take = []
        for req in list(self.pending):
            if len(take) == len(slot.free):
                break
            n = req.hits.shape[0]
            if n > slot.max_hits:
                continue
            # the smallest class that holds the event has priority over this one
            if any(s.max_hits >= n and s.max_hits < slot.max_hits and s.free for s in self.slots):
                continue
            take.append(req)
        if not take:
            return
        for req in take:
            self.pending.remove(req)
        rows = [slot.free.popleft() for _ in take]
        for r, req in zip(rows, take):
            slot.occupant[r] = req
        hits_np = np.concatenate([q.hits for q in take])
        offsets = np.concatenate([[0], np.cumsum([q.hits.shape[0] for q in take])]).astype(np.int32)
        dev = torch.device("cuda", self.device)
        with torch.cuda.stream(slot.stream):
            pinned = torch.from_numpy(hits_np.view(np.float64).reshape(-1, 8).copy()).pin_memory()
            hits = pinned.to(dev, non_blocking=True)
        slot.pool.admit(rows, hits, offsets)
        slot.keep.extend([pinned, hits])

    def _launch(self, slot):
        torch = self.torch
        slot.pool.step()
        ev = torch.cuda.Event()
        ev.record(slot.stream)
        slot.step_ev = ev

    # -- the loop -----------------------------------------------------------
    def run(self, requests, clock=None):
        """Serve `requests` (arrival times in seconds from start).  Returns
        the finished requests with their `done` times set."""
        clock = clock or time.perf_counter
        largest = max(s.max_hits for s in self.slots)
        for r in requests:
            if r.hits.shape[0] > largest:
                raise ValueError(f"request {r.rid} has {r.hits.shape[0]} hits; rows hold at most {largest}")
        t0 = clock()
        now = lambda: clock() - t0  # noqa: E731
        queue = collections.deque(sorted(requests, key=lambda r: r.arrival))
        while queue or self.pending or any(any(o is not None for o in s.occupant) for s in self.slots):
            t = now()
            while queue and queue[0].arrival <= t:
                self.pending.append(queue.popleft())
            idle = True
            for slot in self.slots:
                if slot.busy():
                    idle = False
                    continue
                if slot.step_ev is not None:
                    self._collect(slot, now)
                    slot.step_ev = None
                    slot.keep = []
                self._admit(slot)
                if any(o is not None for o in slot.occupant):
                    self._launch(slot)
                    idle = False
            if idle and queue and not self.pending:
                wait = queue[0].arrival - now()
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            elif not idle:
                time.sleep(20e-6)
        return self.finished

    def close(self):
        for s in self.slots:
            s.pool.close()
            s.ctx.close()


def poisson_arrivals(n, rate, seed=0):
    """n arrival times (s) of a Poisson stream of the given rate (events/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def latency_stats(reqs):
    lat = np.array([r.done - r.arrival for r in reqs])
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "events_per_s": len(reqs) / span}
