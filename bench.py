#!/usr/bin/env python3
"""Benchmark of the interval-arithmetic helix vote on one MI355X.

Workload (one step = one event through the whole search, FP64):
  a single-helix event of the synthetic stereo chamber (20 layers, 0/+60/-60
  mrad superlayers, B = 1 T), drift radii smeared by 150 um, 20 % extra noise
  hits, tolerance band 3 sigma; level-0 grid 16^5 over d0 [-5, 5] mm,
  phi0 [0, 2 pi], kappa [-0.6, 0.6] 1/m, z0 [-5, 5] cm, tanl [-0.8, 0.8];
  four refinement levels, each keeping the 32 max-vote boxes and splitting
  them 4^5; estimate from the max-vote boxes; hit finding.
Each step uses a different seeded event; all hits are resident in HBM
before the timed region.

Prints one JSON line: box-hit evaluations/s (value), events/s, p50/p99 event
latency, the vote kernel's roofline figures and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "box-hit interval evals/s + events/s at 1 GPU; p50/p99 event latency"

# Algorithmic FP64 work of the vote kernel (flops; an FMA counts 2, a division
# or square root 1), counted from the operation sequence of the predicate:
#  - per (box, stereo hit), both drift signs: the stereo virtual drift at the
#    box centre (second-order Phi, sin/cos of its correction, drift-line norm,
#    d^Ax) and the interval test of 2G - 2E - kappa E^2;
#  - per (triple, hit) staged once for all boxes sharing (d0, phi0, kappa):
#    the centre frame, the interval residual G (sin enclosure) and the
#    transverse part of the stereo term (axial hits are decided here).
FLOP_BOX_STEREO = 335
FLOP_TRIPLE_HIT = 310
PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64: 256 CU x 128 FLOP/clk x 2.4 GHz


def level_shapes(bins, top_k, split, n_refine):
    """(n_boxes, n_triples) per level for one helix pass."""
    out = []
    nb0 = int(np.prod(bins))
    out.append((nb0, int(np.prod(bins[:3]))))
    n_par = min(top_k, nb0)
    for _ in range(n_refine):
        nb = n_par * int(np.prod(split))
        out.append((nb, n_par * int(np.prod(split[:3]))))
        n_par = min(top_k, nb)
    return out


def vote_flops(n_boxes, n_triples, n_stereo, n_hits):
    return float(n_boxes) * n_stereo * FLOP_BOX_STEREO + float(n_triples) * n_hits * FLOP_TRIPLE_HIT


def hit_counts(hits):
    dz = hits["z1"] - hits["z0"]
    tx = (hits["x1"] - hits["x0"]) / dz
    ty = (hits["y1"] - hits["y0"]) / dz
    stereo = (tx * tx + ty * ty) > 0
    return int(hits.shape[0]), int(stereo.sum())


def cpu_baseline(events, sched_kw, lo, hi, budget_s=20.0):
    import oracle
    nt = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sched = oracle.make_sched(lo, hi, **sched_kw)
    shapes = level_shapes(sched_kw["bins"], sched_kw["top_k"], sched_kw["split"], sched_kw["n_refine"])
    evals = 0.0
    t0 = time.perf_counter()
    n_done = 0
    for ev in events:
        hel, _ = oracle.find_helices(ev.hits, sched, max_out=1, n_threads=nt)
        n, _ = hit_counts(ev.hits)
        levels = shapes if len(hel) else shapes[:1]
        evals += sum(nb for nb, _ in levels) * n
        n_done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "box-hit evals/s", "cores": nt, "kind": "oracle",
            "sample": f"{n_done} event(s) of the same workload through the whole search "
                      f"(FP64 C oracle, OpenMP over boxes), {dt:.1f} s",
            "events_per_s": n_done / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the search shards by event "
              "across GPUs with no exchange, which this build does not launch.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2401_04576_amd as ia
    from paper_2401_04576_amd import toymc

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    lo, hi = np.array(toymc.GRID_RANGE_LO), np.array(toymc.GRID_RANGE_HI)
    sched_kw = dict(bins=[16] * 5, n_refine=4, top_k=32, split=[4] * 5, v_min=10, n_helix_max=1)
    n_ev = args.warmup + args.steps
    t_gen = time.perf_counter()
    events = [toymc.config_event(2, i) for i in range(n_ev)]
    t_gen = time.perf_counter() - t_gen
    hits_np = np.concatenate([e.hits for e in events])
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])]).astype(np.int64)
    hits = torch.from_numpy(hits_np.view(np.float64).reshape(-1, 8).copy()).to(dev)
    sched = ia.Schedule.make(lo, hi, **sched_kw)
    max_hits = max(e.n_hits for e in events)
    ctx = ia.Context(0, scratch_bytes=ia.Context.scratch_needed(sched, max_hits) + (1 << 20))
    out = torch.zeros(n_ev * ia.HELIX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    n_out = torch.zeros(n_ev, dtype=torch.int32, device=dev)
    assigned = torch.full((hits.shape[0],), -1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    HB = ia.HELIX_DTYPE.itemsize

    def step(i):
        a, b = int(off[i]), int(off[i + 1])
        ia.find_helices(ctx, hits[a:b], [0, b - a], sched, max_per_event=1, stream=stream,
                        out=out[i * HB:(i + 1) * HB], n_out=n_out[i:i + 1], assigned=assigned[a:b])

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    ctx.profile_read()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        step(args.warmup + k)
        ends[k].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_profiling(False)
    n_launch, vote_ms = ctx.profile_read()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    wall = t1 - t0

    # work actually done: a pass stops after level 0 when its max vote is below v_min
    nout = n_out.cpu().numpy()
    shapes = level_shapes(sched_kw["bins"], sched_kw["top_k"], sched_kw["split"], sched_kw["n_refine"])
    evals, flops, launches = 0.0, 0.0, 0
    for k in range(args.steps):
        i = args.warmup + k
        n, n_st = hit_counts(events[i].hits)
        levels = shapes if nout[i] > 0 else shapes[:1]
        for nb, ntr in levels:
            evals += float(nb) * n
            flops += vote_flops(nb, ntr, n_st, n)
            launches += 1
    assert launches == n_launch, (launches, n_launch)
    value = evals / wall
    avg_launch_ms = vote_ms / n_launch
    achieved = flops / n_launch / (avg_launch_ms * 1e-3) / 1e12
    res = {
        "metric": METRIC, "value": value, "unit": "box-hit evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "single event, hierarchical refinement, FP64: 1 helix, 150 um smearing, "
                               "20% noise hits, band 3 sigma; 16^5 level-0 grid then 4 levels of top-32 "
                               "boxes split 4^5; estimate and hit finding",
                   "events": args.steps, "mean_hits": float(np.mean([e.n_hits for e in events[args.warmup:]])),
                   "boxes_per_event": int(sum(nb for nb, _ in shapes))},
        "events_per_s": args.steps / wall,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "kernel": "k_vote", "avg_launch_ms": avg_launch_ms, "launches": n_launch,
                     "vote_share_of_wall": vote_ms * 1e-3 / wall},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(events[args.warmup:], sched_kw, lo, hi, args.cpu_budget)
    ctx.close()
    print(f"[bench] generated {n_ev} events in {t_gen:.1f} s; vote kernel {vote_ms:.2f} ms of "
          f"{wall * 1e3:.2f} ms", file=sys.stderr)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
