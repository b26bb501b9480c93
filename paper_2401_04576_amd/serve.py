"""Continuous-batching serving loop over ia_find_helices.

Events arrive over time (for instance as a Poisson stream).  The loop keeps
`n_slots` execution slots; each slot owns a library context (its scratch
arena, sized from the device-memory budget) and its own stream, so batches
in different slots run concurrently on the device.  Whenever a slot is free,
every event that has arrived and fits the slot's arena is admitted into one
batch and launched; results are collected when the slot's completion event
fires, and each event's latency is measured from its arrival to the moment
its result is back on the host.  An event's result does not depend on the
batch it was served in (the library's kernels treat every event of a batch
independently), which tests/test_gpu_serve.py checks.

The device work itself (prep, votes, selection, estimate, hit finding) runs
in the HIP kernels of libia; this module only schedules host-side work.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import Context, HELIX_DTYPE, Schedule, decode, find_helices


@dataclasses.dataclass
class Request:
    rid: int
    hits: np.ndarray            # structured ia_hit records
    arrival: float              # seconds on the loop's clock
    done: float = float("nan")
    helices: np.ndarray = None  # HELIX_DTYPE records
    assigned: np.ndarray = None


class _Slot:
    def __init__(self, device, scratch_bytes, torch):
        self.ctx = Context(device, scratch_bytes=scratch_bytes)
        self.stream = torch.cuda.Stream(device=device)
        self.done_ev = None
        self.batch = None           # (requests, out, n_out, assigned, offsets)
        self.torch = torch

    def busy(self):
        return self.batch is not None

    def ready(self):
        return self.done_ev is not None and self.done_ev.query()


class ServeLoop:
    """Serve requests with up to `n_slots` concurrent batches.

    scratch_budget: device bytes for all slot arenas together (admission by
    device memory: a batch holds only as many events as its arena fits).
    """

    def __init__(self, sched: Schedule, max_per_event=10, n_slots=4, scratch_budget=8 << 30,
                 max_batch=4096, device=0, max_hits=1000):
        import torch
        self.torch = torch
        self.sched = sched
        self.max_per_event = int(max_per_event)
        self.device = device
        per_slot = int(scratch_budget // n_slots)
        self.per_event_bytes = Context.scratch_needed(sched, max_hits)
        if per_slot < self.per_event_bytes:
            raise ValueError("scratch budget below one event per slot")
        self.events_per_slot = max(1, min(max_batch, per_slot // self.per_event_bytes))
        self.slots = [_Slot(device, per_slot, torch) for _ in range(n_slots)]
        for s in self.slots:
            s.ctx.set_batch(self.events_per_slot)
        self.pending = collections.deque()
        self.finished = []

    # -- batching -----------------------------------------------------------
    def _launch(self, slot: _Slot, reqs):
        torch = self.torch
        dev = torch.device("cuda", self.device)
        hits_np = np.concatenate([r.hits for r in reqs]) if reqs else np.zeros(0)
        offsets = np.concatenate([[0], np.cumsum([r.hits.shape[0] for r in reqs])]).astype(np.int64)
        with torch.cuda.stream(slot.stream):
            pinned = torch.from_numpy(hits_np.view(np.float64).reshape(-1, 8).copy()).pin_memory()
            hits = pinned.to(dev, non_blocking=True)
            n = len(reqs)
            out = torch.empty(n * self.max_per_event * HELIX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
            n_out = torch.empty(n, dtype=torch.int32, device=dev)
            assigned = torch.empty(max(1, hits.shape[0]), dtype=torch.int32, device=dev)
            find_helices(slot.ctx, hits, offsets, self.sched, max_per_event=self.max_per_event,
                         stream=slot.stream, out=out, n_out=n_out, assigned=assigned)
            out_h = out.to("cpu", non_blocking=True)
            n_out_h = n_out.to("cpu", non_blocking=True)
            ass_h = assigned.to("cpu", non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        slot.batch = (reqs, out_h, n_out_h, ass_h, offsets, (pinned, hits, out, n_out, assigned))
        slot.done_ev = ev

    def _collect(self, slot: _Slot, now):
        reqs, out_h, n_out_h, ass_h, offsets, _keep = slot.batch
        hel = decode(out_h, HELIX_DTYPE).reshape(len(reqs), self.max_per_event)
        n_out = n_out_h.numpy()
        ass = ass_h.numpy()
        for i, r in enumerate(reqs):
            r.helices = hel[i, :n_out[i]].copy()
            r.assigned = ass[offsets[i]:offsets[i + 1]].copy()
            r.done = now
            self.finished.append(r)
        slot.batch = None
        slot.done_ev = None

    # -- the loop -----------------------------------------------------------
    def run(self, requests, clock=None):
        """Serve `requests` (sorted by arrival time, seconds from start).
        Returns the finished requests with their `done` times set."""
        clock = clock or time.perf_counter
        t0 = clock()
        queue = collections.deque(sorted(requests, key=lambda r: r.arrival))
        in_flight = 0
        while queue or self.pending or in_flight:
            now = clock() - t0
            while queue and queue[0].arrival <= now:
                self.pending.append(queue.popleft())
            for slot in self.slots:
                if slot.busy() and slot.ready():
                    self._collect(slot, clock() - t0)
                    in_flight -= 1
            for slot in self.slots:
                if not slot.busy() and self.pending:
                    batch = [self.pending.popleft() for _ in range(min(len(self.pending), self.events_per_slot))]
                    self._launch(slot, batch)
                    in_flight += 1
            if not self.pending and queue and not in_flight:
                # idle until the next arrival
                wait = queue[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        return self.finished

    def close(self):
        for s in self.slots:
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
