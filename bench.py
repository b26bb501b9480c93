#!/usr/bin/env python3
"""Benchmark of the interval-arithmetic helix vote on one MI355X.

Workload (one step = one ia_find_helices call over --event-batch events,
default 1024, through the whole search, FP64):
  single-helix events of the synthetic stereo chamber (20 layers,
  0/+60/-60 mrad superlayers, B = 1 T), drift radii smeared by 150 um, 20 %
  extra noise hits, tolerance band 3 sigma; level-0 grid 16^5 over d0
  [-5, 5] mm, phi0 [0, 2 pi], kappa [-0.6, 0.6] 1/m, z0 [-5, 5] cm, tanl
  [-0.8, 0.8]; four refinement levels, each keeping the 32 max-vote boxes
  and splitting them 4^5; estimate from the max-vote boxes; hit finding.
Each step uses different seeded events; all hits are resident in HBM
before the timed region.  p50/p99 are per-event latencies of single-event
calls made after the timed steps.

With --workload batch, one step is instead a batch of 4096 events (1-5
helices, 20-200 hits, 0-30 % noise, the same schedule with up to 5 greedy
helix passes) searched by one ia_find_helices call, whose kernels each cover
every event of a batch.

With --workload mixed-report, noiseless single-helix events go through the
same schedule all in FP64 and with FP32 at levels 0-2: the line reports, per
level, the fraction of boxes whose FP32 and FP64 votes differ on the FP64
frontier's parents, whether the FP32 selection equals the FP64 one, and per
parameter |FP32 - FP64| and |estimate - truth| of the final helices.

With --workload copy, a plain elementwise copy of 1 GiB (torch, float32)
runs a few times: under rocprofv3 --pmc its FETCH_SIZE and WRITE_SIZE per
dispatch against the 1 GiB it moves give the scale of those counters.

With --workload serve, events of the serving mix (1-10 helices, lognormal
hit counts with median 120 clipped to [20, 1000], 0-40 % noise) arrive as a
Poisson stream and are served by the continuous-batching loop; the line
gives p50/p99 arrival-to-result latency and events/s, beside the plain
one-event-per-call FP64 path timed on a sample of the same events.

Prints one JSON line: box-hit evaluations/s (value), events/s, p50/p99 event
latency (per step), the vote kernel's roofline figures and the CPU oracle
baseline.
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
# or square root 1), counted from the operation sequence of the predicate and
# applied to the work counters the library reports:
#  - per stereo (box, hit) evaluation, both drift signs: the stereo virtual
#    drift at the box centre (second-order Phi, sin/cos of its correction,
#    drift-line norm, d^Ax) and the interval test of 2G - 2E - kappa E^2;
#  - per staged (triple, stereo hit) record, shared by the boxes of the
#    triple: the centre frame, the interval residual G (sin enclosure) and
#    the transverse part of the stereo term.
FLOP_BOX_STEREO = 335
FLOP_TRIPLE_HIT = 310
# the same per-box evaluation at FP32 levels (smaller sin/cos polynomials, no
# range reduction), FP32 flops; the staged (triple, hit) work stays FP64
FLOP_BOX_STEREO32 = 278
# (triple, hit) classification, FP64 flops per unit (add, sub, mul, div,
# sqrt 1, fma 2; min, max, abs 0; outward rounding of an end point 3):
#  - residual interval G of a pair (two sin evaluations of the phi0
#    enclosure, the kappa-scaled terms): 157;
#  - axial test, both drift signs (two interval tests of 2G - 2E - kappa E^2): 92;
#  - stereo pair quantities (RAx, its sin / cos, atan2 of the arc, sArc, ...): 69;
#  - one interval enclosure of d^Ax over the triple's (z0, tanl) centres with
#    its exclusion test (the FP32 levels' test counted as FP64 too): 688;
#  - one inclusion proof (bounds at the enclosure's ends): 94;
#  - one magnitude bound of d^Ax over the triple (67) with its exclusion test (46): 113;
#  - a deferred pair's triple frame and (z0, tanl) centre ranges: 130;
#  - the first stage's outer enclosure of G (sines of the phi0 edges from the
#    difference identity, then residual_G's interval operations): 68;
#  - the first stage's stereo pair magnitudes (pair quantities without atan2): 34.
FLOP_CLS_G, FLOP_CLS_AXIAL, FLOP_CLS_PAIRQ, FLOP_CLS_ENCL, FLOP_CLS_INCL, FLOP_CLS_MAG = 157, 92, 69, 688, 94, 113
FLOP_CLS_FRAME, FLOP_CLS_GOUT, FLOP_CLS_PAIRMAG = 130, 68, 34
PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64: 256 CU x 128 FLOP/clk x 2.4 GHz
# Counter record of the default workload's dominant kernel (k_vote_rec over a
# batch of 4,096 config-4 events, all 80 launches of the five full search
# runs: a probe and a vote per level), from rocprofv3 --pmc runs of
# `bench.py --steps 1 --warmup 1 --no-autotune --no-cpu-baseline`
# (profiles/vote_rec_batch4096_window_fp64.md), averaged per launch: HBM
# bytes (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0, the factors that make the
# counters read 1 GiB for a 1 GiB copy) and wave-level FP64 VALU instruction
# counts.  Valid only for the kernel sources and launch shapes they were
# measured on (SHA-256 of ia_math.hpp + ia_kernels.hpp + ia_lib.hip).
TRAFFIC = {"kernel": "k_vote (fp64 levels)", "workload": "batch", "events_per_step": 4096,
           "sources_sha256": "f2fc53e9e838d5ede522355626d95e39504c71b2a0ffc45986de82344029d303",
           "fetch_bytes": 1579480468, "write_bytes": 358304629,
           "valu_f64": {"add": 1.4518e9, "mul": 1.6378e9, "fma": 1.8546e9, "trans": 1.4068e8}, "valu": 6.7779e9}
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 (non-packed)


def prec_text(name):
    return {"fp64": "FP64", "mixed": "FP32 at levels 0-2, FP64 after and the fit",
            "exact": "FP64, the exact Phi of Eq. CSAXtoPHI_a at levels 2 and after",
            "iv": "FP64, d^Ax enclosed over the whole box (sound test) at the last two levels"}[name]


def prec_dtype(name):
    return "f32+f64" if name == "mixed" else "f64"


def sched_prec(name, n_refine):
    """Per-level precision: all FP64; FP32 at levels 0-2 and FP64 after
    (mixed); or FP64 with the exact Phi of Eq. CSAXtoPHI_a at levels 2 and
    after (exact)."""
    import paper_2401_04576_amd as ia
    if name == "fp64":
        return [ia.FP64] * (n_refine + 1)
    if name == "exact":
        return [ia.FP64X if lev >= 2 else ia.FP64 for lev in range(n_refine + 1)]
    if name == "iv":
        return [ia.IV if lev >= n_refine - 1 else ia.FP64 for lev in range(n_refine + 1)]
    return [ia.FP32 if lev <= 2 else ia.FP64 for lev in range(n_refine + 1)]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    # the kernels and their launch shapes (grid sizes live in ia_lib.hip)
    for f in ("ia_math.hpp", "ia_kernels.hpp", "ia_lib.hip"):
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2401_04576_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, events_per_step):
    """(kernel, measured HBM bytes per launch, executed FP64 flops per launch,
    VALU instructions per launch), or None when the workload or the kernel
    sources differ from those of the measurement."""
    t = TRAFFIC
    if workload != t["workload"] or events_per_step != t["events_per_step"]:
        return None
    if kernel_sources_sha256() != t["sources_sha256"]:
        return None
    v = t["valu_f64"]
    flops = 64 * (v["add"] + v["mul"] + 2 * v["fma"] + v["trans"])
    return t["kernel"], t["fetch_bytes"] + t["write_bytes"], flops, t["valu"]


def classify_flops(cw):
    """FP64 flops of the first classification stage."""
    return (cw["G"] * FLOP_CLS_GOUT + cw["axial"] * FLOP_CLS_AXIAL + cw["G_exact"] * (FLOP_CLS_G + FLOP_CLS_AXIAL)
            + cw["pairq"] * FLOP_CLS_PAIRMAG + cw["magnitudes"] * FLOP_CLS_MAG)


def defer_flops(cw):
    """Flops of the second classification stage: FP64 frame, G and pair
    quantities, and the enclosures, which run in FP32 without packed
    instructions, at the same vector rate as FP64."""
    return (cw["deferred"] * (FLOP_CLS_FRAME + FLOP_CLS_G + FLOP_CLS_PAIRQ)
            + cw["enclosures"] * FLOP_CLS_ENCL + cw["inclusions"] * FLOP_CLS_INCL)


def roofline(kprof, work, cwork, wall, measured_on, traffic=None, prec="fp64"):
    """Roofline object of the dominant kernel: of the vote kernel and the
    (triple, hit) classification at FP64 and FP32 levels, the one with the
    largest summed launch time (HIP events around each launch).  Achieved =
    algorithmic flops of the launches / their summed duration; every entry
    is listed under by_kernel."""
    e64, s64, e32, s32 = work
    parts = {}
    n, ms = kprof[("vote", "fp64")]
    if n:
        a = (e64 * FLOP_BOX_STEREO + s64 * FLOP_TRIPLE_HIT) / (ms * 1e-3) / 1e12
        parts["k_vote (fp64 levels)"] = {
            "achieved": a, "peak": PEAK_FP64_TFLOPS, "frac": a / PEAK_FP64_TFLOPS, "avg_launch_ms": ms / n,
            "launches": n, "total_ms": ms, "stereo_box_evals": e64, "staged_pairs": s64}
    n, ms = kprof[("vote", "fp32")]
    if n:
        # FP32 flops of the per-box term only; the FP64 staging is left out
        a = e32 * FLOP_BOX_STEREO32 / (ms * 1e-3) / 1e12
        parts["k_vote (fp32 levels)"] = {
            "achieved": a, "peak": PEAK_FP32_TFLOPS, "frac": a / PEAK_FP32_TFLOPS, "avg_launch_ms": ms / n,
            "launches": n, "total_ms": ms, "stereo_box_evals": e32, "staged_pairs": s32,
            "staged_fp64_tflops": s32 * FLOP_TRIPLE_HIT / (ms * 1e-3) / 1e12}
    for p in ("fp64", "fp32"):
        for kern, fl in (("classify", classify_flops), ("classify_defer", defer_flops)):
            n, ms = kprof[(kern, p)]
            if n:
                a = fl(cwork[p]) / (ms * 1e-3) / 1e12
                parts[f"k_{kern} ({p} levels)"] = {
                    "achieved": a, "peak": PEAK_FP64_TFLOPS, "frac": a / PEAK_FP64_TFLOPS, "avg_launch_ms": ms / n,
                    "launches": n, "total_ms": ms, **cwork[p]}
    dom = max(parts, key=lambda k: parts[k]["total_ms"])
    d = parts[dom]
    executed = None
    if traffic and traffic[0] == dom:
        _, traffic, fl, valu = traffic
        note = "measured on these kernel sources"
        # the counters' executed FP64 flops (64 lanes per wave instruction, an
        # FMA counts 2) and VALU issue over this run's average launch
        sec = d["avg_launch_ms"] * 1e-3
        executed = {"fp64_tflops": fl / sec / 1e12, "frac": fl / sec / 1e12 / PEAK_FP64_TFLOPS,
                    "valu_issue_frac": valu / sec / (256 * 2.4e9),
                    "note": "rocprofv3 SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 and SQ_INSTS_VALU per launch "
                            "(same sources) over this run's average launch; issue peak 1 wave instruction "
                            "per CU per clock, 256 CU x 2.4 GHz"}
    else:
        traffic = None
        note = ("no counter record for this kernel on these kernel sources and this workload "
                f"(the last one covers {TRAFFIC['kernel']} on sources {TRAFFIC['sources_sha256'][:12]})")
    return {"bound": "alu", "achieved": d["achieved"], "peak": d["peak"], "unit": "TFLOP/s", "frac": d["frac"],
            "traffic": traffic, "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
            "traffic_note": note, "executed": executed,
            "kernel": dom, "avg_launch_ms": d["avg_launch_ms"], "launches": d["launches"],
            "share_of_wall": d["total_ms"] * 1e-3 / wall, "measured_on": measured_on,
            "by_kernel": parts,
            **({"levels_note": "the fp64-levels record covers every level that is not FP32 (FP64, exact-Phi and "
                               "whole-box levels); its algorithmic flops count the mid-voxel test's, so it "
                               "understates the exact-Phi and whole-box kernels' work"}
               if prec in ("exact", "iv") else {})}


def kernel_measure(ctx, run):
    """Per-kernel launch durations (HIP events on the launch stream around
    every vote and classification launch) over one run of `run`, the vote
    kernel's work counters of that run, then the classification's work over
    a second, counting run of the same work (the search is deterministic).
    Both runs follow the timed region, which carries no events or counters."""
    import torch
    torch.cuda.synchronize()
    ctx.profile_kernels()
    ctx.clear_status()
    ctx.set_profiling(True)
    try:
        run()
        torch.cuda.synchronize()
    finally:
        ctx.set_profiling(False)
    kprof = ctx.profile_kernels()
    work = ctx.work()
    ctx.clear_status()
    ctx.set_work_counting(True)
    try:
        run()
        torch.cuda.synchronize()
    finally:
        ctx.set_work_counting(False)
    return kprof, work, ctx.classify_work()


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


def hit_counts(hits):
    dz = hits["z1"] - hits["z0"]
    tx = (hits["x1"] - hits["x0"]) / dz
    ty = (hits["y1"] - hits["y0"]) / dz
    stereo = (tx * tx + ty * ty) > 0
    return int(hits.shape[0]), int(stereo.sum())


def event_evals(n_valid, helices, n_out, shapes, n_helix_max):
    """Box-hit evaluations of one event, from its recorded helices: every
    recorded helix is a full pass over the hits still active; a pass that
    stops at level 0 (maximum below v_min) adds level 0 only."""
    full = sum(nb for nb, _ in shapes)
    active, ev = n_valid, 0.0
    for h in range(n_out):
        ev += full * active
        active -= int(helices[h]["n_assigned"])
    if n_out < n_helix_max and (n_out == 0 or int(helices[n_out - 1]["n_assigned"]) > 0):
        ev += shapes[0][0] * active
    return ev


def window_shapes(sched_kw):
    """(n_boxes, n_triples) per level of the window schedule (one window per level)."""
    out = [(int(np.prod(sched_kw["bins"])), int(np.prod(sched_kw["bins"][:3])))]
    for lev in range(1, sched_kw["n_refine"] + 1):
        b = sched_kw["lbins"][lev]
        out.append((int(np.prod(b)), int(np.prod(b[:3]))))
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_level0(events, sched_kw, lo, hi, budget_s=20.0):
    """The oracle timed on the host: the level-0 vote (every box of the 16^5
    grid against every hit, with the forward-hit test of the schedule) of the
    first events of the batch, on all threads, and on one thread over the first
    1/16 of the boxes.  The oracle evaluates every (box, hit) pair on its own,
    so its rate is in interval evaluations per second."""
    import oracle
    nt = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    grid = oracle.make_box(lo, hi)
    bins = list(sched_kw["bins"])
    fwd = bool(sched_kw.get("forward", False))
    pairs, n_done = 0.0, 0
    t0 = time.perf_counter()
    for ev in events:
        oracle.vote_level(ev.hits, grid, bins, n_threads=nt, forward=fwd)
        pairs += float(np.prod(bins)) * ev.n_hits
        n_done += 1
        if time.perf_counter() - t0 > budget_s * 0.75:
            break
    dt = time.perf_counter() - t0
    # one thread: the first 1/16 of the boxes (the slowest index split by 16)
    sub = oracle.make_box(lo, hi)
    sub["hi"][0] = lo[0] + (hi[0] - lo[0]) / 16.0
    b1 = [1] + bins[1:]
    t1 = time.perf_counter()
    oracle.vote_level(events[0].hits, sub, b1, n_threads=1, forward=fwd)
    dt1 = time.perf_counter() - t1
    p1 = float(np.prod(b1)) * events[0].n_hits
    return {"value": pairs / dt, "unit": "box-hit interval evals/s", "cores": nt, "kind": "oracle",
            "sample": f"level-0 vote of {n_done} event(s) of the timed batch (16^5 boxes x their hits, "
                      f"{pairs:.3g} pairs) on {nt} threads in {dt:.1f} s",
            "one_thread": {"value": p1 / dt1, "sample": f"1/16 of event 0's level-0 boxes, {dt1:.1f} s"},
            "cpu_model": cpu_model()}


def _gen(args):
    cfg, i = args
    from paper_2401_04576_amd import toymc
    return toymc.config_event(cfg, i)


def generate(cfg, indices):
    indices = list(indices)
    if len(indices) < 64:
        return [_gen((cfg, i)) for i in indices]
    import multiprocessing as mp
    # close and join (not terminate) the workers, so that none is killed
    # while a profiler is attached to this process
    pool = mp.get_context("fork").Pool(min(16, os.cpu_count() or 1))
    try:
        out = pool.map(_gen, [(cfg, i) for i in indices], chunksize=16)
    finally:
        pool.close()
        pool.join()
    return out


def cpu_baseline(events, sched_kw, lo, hi, budget_s=20.0):
    import oracle
    nt = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sched = oracle.make_sched(lo, hi, **sched_kw)
    shapes = level_shapes(sched_kw["bins"], sched_kw["top_k"], sched_kw["split"], sched_kw["n_refine"])
    evals = 0.0
    t0 = time.perf_counter()
    n_done = 0
    nh = sched_kw["n_helix_max"]
    for ev in events:
        hel, _ = oracle.find_helices(ev.hits, sched, max_out=nh, n_threads=nt)
        n, _ = hit_counts(ev.hits)
        evals += event_evals(n, hel, len(hel), shapes, nh)
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
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--workload", choices=["event", "batch", "serve", "mixed-report", "copy"], default="batch")
    ap.add_argument("--sched", choices=["window", "topk"], default="window",
                    help="window: re-gridding from all max-vote boxes with a moved reference point (recovers "
                         "helices); topk: 16^5 then 4 levels of the top-32 boxes split 4^5 (the literal schedule)")
    ap.add_argument("--batch-events", type=int, default=4096)
    ap.add_argument("--event-batch", type=int, default=1024,
                    help="single-helix workload: events per ia_find_helices call (one step)")
    ap.add_argument("--latency-events", type=int, default=40,
                    help="single-helix workload: single-event calls timed for p50/p99 latency")
    ap.add_argument("--scratch-gb", type=float, default=48.0)
    ap.add_argument("--serve-events", type=int, default=2048)
    ap.add_argument("--serve-rows", type=int, default=256, help="serving: rows per pool at most")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serving: Poisson arrival rate, events/s (0: 0.8 x the measured saturated rate)")
    ap.add_argument("--report-events", type=int, default=1000, help="mixed-report: noiseless single-helix events")
    ap.add_argument("--no-autotune", action="store_true", help="skip the vote-tile autotuner")
    ap.add_argument("--no-graph", action="store_true",
                    help="batch: call ia_find_helices per step instead of replaying a captured graph")
    ap.add_argument("--prec", choices=["fp64", "mixed", "exact", "iv"], default="fp64",
                    help="mixed: FP32 vote arithmetic at levels 0-2, FP64 at the finer levels and the fit; "
                         "exact: the exact Phi of Eq. CSAXtoPHI_a at levels 2 and after; iv: d^Ax enclosed "
                         "over the whole box at the last two levels")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the search shards by event "
              "across GPUs with no exchange, which this build does not launch.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2401_04576_amd as ia
    from paper_2401_04576_amd import toymc

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "mixed-report":
        return run_mixed_report(args)
    if args.workload == "copy":
        return run_copy(args)
    return run_event(args)


def run_copy(args):
    """Calibration of the HBM traffic counters: an elementwise copy that
    reads and writes exactly 1 GiB per dispatch."""
    import torch
    n = (1 << 30) // 4
    x = torch.rand(n, device="cuda:0", dtype=torch.float32)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    assert torch.equal(x, y)
    print(json.dumps({"workload": "copy", "bytes_read_per_dispatch": n * 4, "bytes_written_per_dispatch": n * 4,
                      "dispatches": reps, "ms_per_dispatch": dt * 1e3, "GBps": 2 * n * 4 / dt / 1e9}), flush=True)


def run_event(args):
    """The single-helix workload (16^5 grid, 4 refinement levels, FP64 or
    mixed): each step is one ia_find_helices call over --event-batch events;
    then single-event calls give the per-event latency."""
    import torch

    import paper_2401_04576_amd as ia
    from paper_2401_04576_amd import toymc

    dev = torch.device("cuda:0")
    lo, hi = np.array(toymc.GRID_RANGE_LO), np.array(toymc.GRID_RANGE_HI)
    sched_kw = dict(bins=[16] * 5, n_refine=4, top_k=32, split=[4] * 5, v_min=10, n_helix_max=1)
    prec = sched_prec(args.prec, sched_kw["n_refine"])
    B = max(1, args.event_batch)
    n_lat = args.latency_events
    n_ev = (args.warmup + args.steps) * B + n_lat
    t_gen = time.perf_counter()
    events = generate(2, range(n_ev))
    t_gen = time.perf_counter() - t_gen
    sched = ia.Schedule.make(lo, hi, prec=prec, **sched_kw)
    max_hits = max(e.n_hits for e in events)
    per_event = ia.Context.scratch_needed(sched, max_hits)
    ctx = ia.Context(0, scratch_bytes=min(int(args.scratch_gb * (1 << 30)), per_event * B * 2) + (16 << 20))
    HB = ia.HELIX_DTYPE.itemsize
    stream = torch.cuda.current_stream()
    batches = []
    for k in range(args.warmup + args.steps):
        evs = events[k * B:(k + 1) * B]
        h = np.concatenate([e.hits for e in evs])
        off = np.concatenate([[0], np.cumsum([e.n_hits for e in evs])]).astype(np.int64)
        batches.append((evs, torch.from_numpy(h.view(np.float64).reshape(-1, 8).copy()).to(dev), off,
                        torch.zeros(B * HB, dtype=torch.uint8, device=dev),
                        torch.zeros(B, dtype=torch.int32, device=dev),
                        torch.full((h.shape[0],), -1, dtype=torch.int32, device=dev)))

    tuned = {} if args.no_autotune else ctx.autotune(batches[0][1], batches[0][2], sched, max_per_event=1)

    def step(k):
        evs, hits, off, out, n_out, assigned = batches[k]
        ia.find_helices(ctx, hits, off, sched, max_per_event=1, stream=stream, out=out, n_out=n_out,
                        assigned=assigned)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        step(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kprof, work, cwork = kernel_measure(ctx, lambda: [step(k) for k in range(args.warmup, args.warmup + args.steps)])

    # work of the schedule: a pass that stops at level 0 (maximum below
    # v_min) has level 0 only
    shapes = level_shapes(sched_kw["bins"], sched_kw["top_k"], sched_kw["split"], sched_kw["n_refine"])
    evals, found = 0.0, 0
    for k in range(args.warmup, args.warmup + args.steps):
        evs, _, _, _, n_out, _ = batches[k]
        nout = n_out.cpu().numpy()
        for e, ev in enumerate(evs):
            n, _ = hit_counts(ev.hits)
            levels = shapes if nout[e] > 0 else shapes[:1]
            evals += sum(float(nb) * n for nb, _ in levels)
            found += int(nout[e])

    # per-event latency: single-event calls, each timed on its own
    lat = []
    if n_lat:
        lat_evs = events[(args.warmup + args.steps) * B:]
        hl = [torch.from_numpy(e.hits.view(np.float64).reshape(-1, 8).copy()).to(dev) for e in lat_evs]
        o1 = torch.zeros(HB, dtype=torch.uint8, device=dev)
        n1 = torch.zeros(1, dtype=torch.int32, device=dev)
        for i, h in enumerate(hl):
            a1 = torch.full((h.shape[0],), -1, dtype=torch.int32, device=dev)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            ia.find_helices(ctx, h, [0, h.shape[0]], sched, max_per_event=1, stream=stream, out=o1, n_out=n1,
                            assigned=a1)
            torch.cuda.synchronize()
            if i >= 3:
                lat.append((time.perf_counter() - ts) * 1e3)
    n_done = B * args.steps
    res = {
        "metric": METRIC, "value": evals / wall, "unit": "box-hit evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec_dtype(args.prec),
        "data": "synthetic",
        "config": {"workload": f"single-helix events, {B} per ia_find_helices call, hierarchical refinement, "
                               + prec_text(args.prec)
                               + ": 20 layers, 150 um smearing, 20% noise hits, band 3 sigma; 16^5 level-0 grid "
                               "then 4 levels of top-32 boxes split 4^5; estimate and hit finding",
                   "events_per_step": B, "mean_hits": float(np.mean([e.n_hits for e in events])),
                   "boxes_per_event": int(sum(nb for nb, _ in shapes)),
                   "helices_found_per_event": found / n_done,
                   "vote_tiles": {str(k): v for k, v in tuned.items()}},
        "events_per_s": n_done / wall,
        "p50_ms": float(np.percentile(lat, 50)) if lat else None,
        "p99_ms": float(np.percentile(lat, 99)) if lat else None,
        "latency": "p50/p99: one event per call, arrival of resident hits to its recorded helix",
        "roofline": roofline(kprof, work, cwork, wall,
                             "repeat of the timed steps: HIP events around each launch, then a work-counting run",
                             measured_traffic("event", B), args.prec),
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(batches[args.warmup][0], sched_kw, lo, hi, args.cpu_budget)
    ctx.close()
    print(f"[bench] generated {n_ev} events in {t_gen:.1f} s; vote kernel "
          f"{kprof[('vote', 'fp64')][1] + kprof[('vote', 'fp32')][1]:.2f} ms, classification "
          f"{kprof[('classify', 'fp64')][1] + kprof[('classify', 'fp32')][1]:.2f} ms of {wall * 1e3:.2f} ms",
          file=sys.stderr)
    print(json.dumps(res), flush=True)


def schedule_kw(name, n_helix_max):
    from paper_2401_04576_amd import toymc
    kw = dict(toymc.WINDOW_KW if name == "window" else toymc.TOPK_KW)
    kw.update(v_min=10, n_helix_max=n_helix_max)
    return kw


def schedule_text(name):
    if name == "window":
        return ("window schedule: 16^5 grid, a 16^5 window on all max-vote boxes, reference point moved to the "
                "hit closest to the estimate, six 12^5 windows; forward-hit test before the move; per-level hit "
                "selection")
    return "top-k schedule: 16^5 grid then 4 levels of the top-32 boxes split 4^5"


def recovery(evs, hel, nout):
    """Generated helices recovered within the tolerances by a found helix
    that assigned hits; found helices matching none (fakes)."""
    from paper_2401_04576_amd import toymc
    rec = tot = fake = found = rec_t = 0
    for e, ev in enumerate(evs):
        f = hel[e, :int(nout[e])]
        f = f[f["n_assigned"] > 0]
        m = toymc.match_helices(f["p"], ev.truth)
        mt = toymc.match_helices(f["p"], ev.truth, toymc.TRANSVERSE_TOL)
        found += len(f)
        fake += int((m < 0).sum())
        rec += len(set(int(x) for x in m if x >= 0))
        rec_t += len(set(int(x) for x in mt if x >= 0))
        tot += len(ev.truth)
    return {"recovered": rec, "generated": tot, "rate": rec / max(tot, 1), "found": found, "unmatched": fake,
            "recovered_transverse": rec_t}


def performed_evals(work, cwork):
    """Interval evaluations of Eq. ApoVote the library performed: one per
    live (triple, hit) pair classified over its whole triple, and one per
    (box, stereo hit) pair evaluated box by box."""
    e64, _, e32, _ = work
    return cwork["fp64"]["G"] + cwork["fp32"]["G"] + e64 + e32


def run_batch(args):
    """Workload 4: batches of events through one ia_find_helices call each."""
    import torch

    import paper_2401_04576_amd as ia
    from paper_2401_04576_amd import toymc

    dev = torch.device("cuda:0")
    lo, hi = np.array(toymc.GRID_RANGE_LO), np.array(toymc.GRID_RANGE_HI)
    nh = 5
    sched_kw = schedule_kw(args.sched, nh)
    prec = sched_prec(args.prec, sched_kw["n_refine"])
    E = args.batch_events
    n_batches = args.warmup + args.steps
    t_gen = time.perf_counter()
    events = generate(4, range(E * n_batches))
    t_gen = time.perf_counter() - t_gen
    sched = ia.Schedule.make(lo, hi, prec=prec, **sched_kw)
    ctx = ia.Context(0, scratch_bytes=int(args.scratch_gb * (1 << 30)))
    batches = []
    for b in range(n_batches):
        evs = events[b * E:(b + 1) * E]
        hits_np = np.concatenate([e.hits for e in evs])
        off = np.concatenate([[0], np.cumsum([e.n_hits for e in evs])]).astype(np.int64)
        hits = torch.from_numpy(hits_np.view(np.float64).reshape(-1, 8).copy()).to(dev)
        out = torch.zeros(E * nh * ia.HELIX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        n_out = torch.zeros(E, dtype=torch.int32, device=dev)
        assigned = torch.full((hits.shape[0],), -1, dtype=torch.int32, device=dev)
        batches.append((evs, hits, off, out, n_out, assigned))
    stream = torch.cuda.current_stream()
    tuned = {} if args.no_autotune else ctx.autotune(batches[0][1], batches[0][2], sched, max_per_event=nh)
    use_graph = not args.no_graph
    if use_graph:
        # one capture of the device-offset search over static buffers sized for
        # E events of the workload's largest hit count; each step copies its
        # batch in and replays the graph
        max_h = 200
        static_hits = torch.zeros((E * max_h, 8), dtype=torch.float64, device=dev)
        static_off = torch.zeros(E + 1, dtype=torch.int32, device=dev)
        d_offs = [torch.from_numpy(b[2].astype(np.int32)).to(dev) for b in batches]
        g_out = torch.zeros(E * nh * ia.HELIX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        g_nout = torch.zeros(E, dtype=torch.int32, device=dev)
        g_ass = torch.full((E * max_h,), -1, dtype=torch.int32, device=dev)
        cap = torch.cuda.Stream()
        ia.find_helices_dev(ctx, static_hits, static_off, max_h, sched, g_out, g_nout, g_ass, max_per_event=nh,
                            stream=cap)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=cap):
            ia.find_helices_dev(ctx, static_hits, static_off, max_h, sched, g_out, g_nout, g_ass, max_per_event=nh,
                                stream=cap)
        torch.cuda.synchronize()

    def step(b):
        evs, hits, off, out, n_out, assigned = batches[b]
        if use_graph:
            static_hits[:hits.shape[0]].copy_(hits)
            static_off.copy_(d_offs[b])
            graph.replay()
            out.copy_(g_out)
            n_out.copy_(g_nout)
            assigned.copy_(g_ass[:hits.shape[0]])
        else:
            ia.find_helices(ctx, hits, off, sched, max_per_event=nh, stream=stream, out=out, n_out=n_out,
                            assigned=assigned)

    for b in range(args.warmup):
        step(b)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        step(args.warmup + k)
        ends[k].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    wall = t1 - t0
    if use_graph:
        # a captured graph holds no per-launch timing events: launch durations
        # and work come from an eager repeat of the last timed batch (the same
        # kernels on the same events)
        evs, hits, off, out, n_out, assigned = batches[args.warmup + args.steps - 1]

        def rerun():
            ia.find_helices(ctx, hits, off, sched, max_per_event=nh, stream=stream, out=torch.empty_like(out),
                            n_out=torch.empty_like(n_out), assigned=torch.empty_like(assigned))
        rep_steps = 1
    else:
        def rerun():
            for k in range(args.steps):
                step(args.warmup + k)
        rep_steps = args.steps
    kprof, work, cwork = kernel_measure(ctx, rerun)
    # interval evaluations performed in the timed steps: the work counters
    # over an eager counting repeat of every timed batch (deterministic, so
    # the same work as the replays)
    torch.cuda.synchronize()
    ctx.clear_status()
    ctx.set_work_counting(True)
    try:
        for k in range(args.steps):
            evs, hits, off, out, n_out, assigned = batches[args.warmup + k]
            ia.find_helices(ctx, hits, off, sched, max_per_event=nh, stream=stream, out=torch.empty_like(out),
                            n_out=torch.empty_like(n_out), assigned=torch.empty_like(assigned))
        torch.cuda.synchronize()
    finally:
        ctx.set_work_counting(False)
    evals = performed_evals(ctx.work(), ctx.classify_work())
    shapes = window_shapes(sched_kw) if args.sched == "window" else level_shapes(
        sched_kw["bins"], sched_kw["top_k"], sched_kw["split"], sched_kw["n_refine"])
    nominal, found, truth = 0.0, 0, 0
    recs = []
    for k in range(args.steps):
        evs, hits, off, out, n_out, assigned = batches[args.warmup + k]
        hel = ia.decode(out, ia.HELIX_DTYPE).reshape(E, nh)
        nout = n_out.cpu().numpy()
        recs.append(recovery(evs, hel, nout))
        for e, ev in enumerate(evs):
            n, _ = hit_counts(ev.hits)
            nominal += event_evals(n, hel[e], int(nout[e]), shapes, nh)
            found += int(nout[e])
            truth += ev.truth.shape[0]
    rec = {k: sum(r[k] for r in recs) for k in ("recovered", "generated", "found", "unmatched", "recovered_transverse")}
    rec["rate"] = rec["recovered"] / max(rec["generated"], 1)
    rec["rate_transverse"] = rec["recovered_transverse"] / max(rec["generated"], 1)
    rec["tolerances"] = ("|d0| 1 mm, |phi0| 5 mrad, |kappa| 0.01 /m, |z0| 10 mm, |tanl| 0.02; transverse: the first "
                         "three only; a generated helix counts once")
    res = {
        "metric": METRIC, "value": evals / wall, "unit": "box-hit interval evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec_dtype(args.prec), "data": "synthetic",
        "config": {"workload": f"batched: {E} events per "
                               + ("replay of one captured ia_find_helices_dev graph" if use_graph
                                  else "ia_find_helices call") + ", 1-5 helices and 20-200 hits "
                               "per event, 0-30% noise, 150 um smearing, band 3 sigma; "
                               + schedule_text(args.sched) + "; up to 5 greedy helix passes; "
                               + prec_text(args.prec),
                   "events_per_step": E, "helices_found_per_event": found / (E * args.steps),
                   "vote_tiles": {str(k): v for k, v in tuned.items()},
                   "helices_generated_per_event": truth / (E * args.steps)},
        "value_counts": "interval evaluations of Eq. ApoVote performed: live (triple, hit) pairs classified "
                        "over their whole triple plus (box, stereo hit) pairs evaluated box by box",
        "interval_evals_per_step": evals / args.steps,
        "nominal_box_hit_pairs_per_s": nominal / wall,
        "nominal_counts": "boxes of every level x the hits active in the pass (each is decided, most in bulk)",
        "events_per_s": E * args.steps / wall,
        "recovery": rec,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "latency": "p50/p99 of the step (one batch of events, resident hits to recorded helices)",
        "roofline": roofline(kprof, work, cwork, wall * rep_steps / args.steps,
                             ("eager repeat of the last timed batch" if use_graph else "repeat of the timed steps")
                             + ": HIP events around each launch, then a work-counting run",
                             measured_traffic("batch", E), args.prec),
    }
    if use_graph:
        res["roofline"]["measured_on"] = "eager profiled repeat of the last timed batch"
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_level0(batches[args.warmup][0], sched_kw, lo, hi, args.cpu_budget)
    ctx.close()
    print(f"[bench] generated {len(events)} events in {t_gen:.1f} s", file=sys.stderr)
    print(json.dumps(res), flush=True)


def run_serve(args):
    """Workload 5: config-5 events served by resident pools (continuous
    batching at helix-pass granularity).  First the saturated rate (every
    event waiting at the start), then Poisson arrivals at --rate, or at 0.8x
    the saturated rate when --rate is 0, with p50/p99 from arrival to result;
    beside it the plain FP64 path, one ia_find_helices call per event, on a
    sample of the same events (the same results, so the same recovery)."""
    import torch

    import paper_2401_04576_amd as ia
    from paper_2401_04576_amd import serve, toymc

    dev = torch.device("cuda:0")
    lo, hi = np.array(toymc.GRID_RANGE_LO), np.array(toymc.GRID_RANGE_HI)
    nh = 10
    sched_kw = schedule_kw("window", nh)
    sched = ia.Schedule.make(lo, hi, prec=sched_prec(args.prec, sched_kw["n_refine"]), **sched_kw)
    n_warm = min(256, args.serve_events)
    t_gen = time.perf_counter()
    events = generate(5, range(2 * args.serve_events + n_warm))
    t_gen = time.perf_counter() - t_gen
    warm, sat_events, events = events[:n_warm], events[n_warm:n_warm + args.serve_events], \
        events[n_warm + args.serve_events:]
    loop = serve.ServeLoop(sched, max_per_event=nh, scratch_budget=int(args.scratch_gb * (1 << 30)),
                           rows_cap=args.serve_rows)
    loop.run([serve.Request(i, e.hits, 0.0) for i, e in enumerate(warm)])
    loop.finished = []
    torch.cuda.synchronize()
    # saturation: every event waiting at the start
    t0 = time.perf_counter()
    loop.run([serve.Request(i, e.hits, 0.0) for i, e in enumerate(sat_events)])
    torch.cuda.synchronize()
    sat_rate = len(sat_events) / (time.perf_counter() - t0)
    loop.finished = []
    rate = args.rate if args.rate > 0 else 0.8 * sat_rate
    arrivals = serve.poisson_arrivals(len(events), rate, seed=11)
    reqs = [serve.Request(i, e.hits, float(t)) for i, (e, t) in enumerate(zip(events, arrivals))]
    t0 = time.perf_counter()
    done = loop.run(reqs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    caps = loop.capacity()
    loop.close()
    st = serve.latency_stats(done)
    done.sort(key=lambda r: r.rid)
    hel = np.zeros((len(done), nh), dtype=ia.HELIX_DTYPE)
    nout = np.zeros(len(done), dtype=np.int32)
    for k, r in enumerate(done):
        nout[k] = len(r.helices)
        hel[k, :nout[k]] = r.helices
    rec = recovery(events, hel, nout)

    # the plain FP64 one-event-per-call path on a sample of the same events
    n_plain = min(len(events), 256)
    ctx = ia.Context(0, scratch_bytes=ia.Context.scratch_needed(sched, 1000) + (1 << 20))
    plain_hits = [torch.from_numpy(e.hits.view(np.float64).reshape(-1, 8).copy()).to(dev) for e in events[:n_plain]]
    torch.cuda.synchronize()
    for h in plain_hits[:8]:
        ia.find_helices(ctx, h, [0, h.shape[0]], sched, max_per_event=nh)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat_plain = []
    same = 0
    for k, h in enumerate(plain_hits):
        ta = time.perf_counter()
        raw, n_o, _ = ia.find_helices(ctx, h, [0, h.shape[0]], sched, max_per_event=nh)
        torch.cuda.synchronize()
        lat_plain.append(time.perf_counter() - ta)
        n1 = int(n_o.cpu()[0])
        same += int(ia.decode(raw, ia.HELIX_DTYPE)[:n1].tobytes() == done[k].helices.tobytes())
    plain_wall = time.perf_counter() - t1
    ctx.close()
    res = {
        "metric": METRIC, "value": len(done) / wall, "unit": "events/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec_dtype(args.prec), "data": "synthetic",
        "config": {"workload": f"serving: {len(events)} config-5 events (1-10 helices, lognormal hits median 120 in "
                               f"[20, 1000], 0-40% noise), Poisson arrivals at {rate:.0f}/s; resident pools "
                               "(continuous batching per helix pass) of rows of 128/256/512/1024 hits; window "
                               "schedule, up to 10 greedy helix passes; "
                               + prec_text(args.prec),
                   "rows": caps, "helices_found_per_event": float(nout.mean()),
                   "helices_generated_per_event": float(np.mean([len(e.truth) for e in events]))},
        "saturated_events_per_s": sat_rate, "offered_rate": rate, "rate_rule": "0.8 x saturated" if args.rate <= 0
        else "given", "events_per_s": len(done) / wall,
        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
        "latency": "arrival to result on the host",
        "recovery": rec,
        "plain_fp64_per_event": {"events_per_s": n_plain / plain_wall,
                                 "p50_ms": float(np.percentile(lat_plain, 50) * 1e3),
                                 "p99_ms": float(np.percentile(lat_plain, 99) * 1e3), "events": n_plain,
                                 "same_helices_as_served": same},
    }
    print(f"[bench] generated {len(events) + len(sat_events) + n_warm} events in {t_gen:.1f} s", file=sys.stderr)
    print(json.dumps(res), flush=True)


def run_mixed_report(args):
    """FP32 coarse levels against all-FP64 on noiseless single-helix events
    (config 3), under the window schedule: the votes of the level-0 grid and
    of a 16^5 window around its max-vote boxes both ways (disagreement,
    superset, maximum and max-vote set agreement), then the whole search
    both ways (helix differences and recovery)."""
    import torch

    import paper_2401_04576_amd as ia
    from paper_2401_04576_amd import toymc

    dev = torch.device("cuda:0")
    lo, hi = np.array(toymc.GRID_RANGE_LO), np.array(toymc.GRID_RANGE_HI)
    kw = schedule_kw("window", 1)
    prec_mixed = sched_prec("mixed", kw["n_refine"])
    n = args.report_events
    t_gen = time.perf_counter()
    events = generate(3, range(n))
    t_gen = time.perf_counter() - t_gen
    ctx = ia.Context(0, scratch_bytes=int(args.scratch_gb * (1 << 30)))
    t0 = time.perf_counter()

    # 1. two grids per event: the level-0 grid over the range, and a 16^5
    #    window over the FP64 max-vote boxes widened by one bin
    names_l = ["level 0 (16^5 over the range)", "16^5 window around the level-0 max-vote boxes"]
    diff = np.zeros(2)
    tot = np.zeros(2)
    superset_ok = [True, True]
    max_agree = np.zeros(2)
    set_agree = np.zeros(2)
    root = torch.tensor([list(lo) + list(hi)], dtype=torch.float64, device=dev)
    m = np.array(kw["bins"])
    for ev in events:
        hits = torch.from_numpy(ev.hits.view(np.float64).reshape(-1, 8).copy()).to(dev)
        parents = root
        for g in range(2):
            v64 = ia.vote_level(ctx, hits, parents, kw["bins"], prec=ia.FP64).cpu().numpy().astype(np.int64)
            v32 = ia.vote_level(ctx, hits, parents, kw["bins"], prec=ia.FP32).cpu().numpy().astype(np.int64)
            d = v32 - v64
            diff[g] += np.count_nonzero(d)
            tot[g] += d.size
            superset_ok[g] &= bool(d.min() >= 0)
            max_agree[g] += bool(v64.max() == v32.max())
            set_agree[g] += bool(np.array_equal(np.flatnonzero(v64 == v64.max()), np.flatnonzero(v32 == v32.max())))
            if g == 0:
                p = parents.cpu().numpy()[0]
                plo, phi_ = p[:5], p[5:]
                w = (phi_ - plo) / m
                idx = np.array(np.unravel_index(np.flatnonzero(v64 == v64.max()), tuple(m))).T
                wlo = plo + (idx.min(axis=0) - 1) * w
                whi = plo + (idx.max(axis=0) + 2) * w
                parents = torch.tensor([list(wlo) + list(whi)], dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    # 2. the whole search both ways, batched: final helices
    hits_np = np.concatenate([e.hits for e in events])
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])]).astype(np.int64)
    hits = torch.from_numpy(hits_np.view(np.float64).reshape(-1, 8).copy()).to(dev)
    res_h = {}
    for name, prec in (("fp64", None), ("mixed", prec_mixed)):
        sched = ia.Schedule.make(lo, hi, prec=prec, **kw)
        raw, n_out, _ = ia.find_helices(ctx, hits, off, sched, max_per_event=1)
        torch.cuda.synchronize()
        res_h[name] = (ia.decode(raw, ia.HELIX_DTYPE).reshape(n, 1), n_out.cpu().numpy())
    ctx.close()
    h64, n64 = res_h["fp64"]
    h32, n32 = res_h["mixed"]
    both = (n64 > 0) & (n32 > 0)
    names = ["d0", "phi0", "kappa", "z0", "tanl"]

    def wrap(x):
        return (x + np.pi) % (2 * np.pi) - np.pi

    def stats(x):
        x = np.abs(x)
        return {"mean": float(x.mean()), "rms": float(np.sqrt((x * x).mean())), "max": float(x.max())} if x.size else None

    dpar = {}
    for j, nm in enumerate(names):
        a, b = h32[both, 0]["p"][:, j], h64[both, 0]["p"][:, j]
        dpar[nm] = stats(wrap(a - b) if j == 1 else a - b)
    same = int(sum(h32[e, 0].tobytes() == h64[e, 0].tobytes() for e in range(n) if both[e]))
    res = {
        "metric": METRIC, "value": None, "unit": "report", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": (t1 - t0) * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"FP32 at levels 0-2 (the whole predicate in FP32) against all-FP64: {n} noiseless "
                               "single-helix events, window schedule, band 0"},
        "grids": [{"grid": names_l[g], "vote_disagreement": float(diff[g] / tot[g]),
                   "fp32_votes_contain_fp64": bool(superset_ok[g]), "max_agreement": float(max_agree[g] / n),
                   "max_set_agreement": float(set_agree[g] / n)} for g in range(2)],
        "helices_both": int(both.sum()), "identical_helices": same,
        "abs_fp32_minus_fp64": dpar,
        "recovery_fp64": recovery(events, h64, n64), "recovery_mixed": recovery(events, h32, n32),
    }
    print(f"[bench] generated {n} events in {t_gen:.1f} s", file=sys.stderr)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
