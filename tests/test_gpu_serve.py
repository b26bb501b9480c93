"""Serving loop: continuous batching over several slots gives every event the
result it gets alone, and that result matches the oracle.

Events of the serving mix (1-10 helices, lognormal hit counts, 0-40 % noise)
arrive as a Poisson stream fast enough that batches of different sizes form
and overlap on the device.
"""
import numpy as np
import pytest

import oracle
import paper_2401_04576_amd as ia
from paper_2401_04576_amd import serve, toymc
from tests import _helpers as H

pytestmark = pytest.mark.gpu

KW = dict(bins=[8] * 5, n_refine=2, top_k=16, split=[2] * 5, v_min=10, n_helix_max=4)


def _solo(ctx, ev, sched, nh):
    import torch
    hits = torch.from_numpy(np.ascontiguousarray(ev.hits).view(np.float64).reshape(-1, 8).copy()).to("cuda:0") \
        if ev.n_hits else torch.zeros((0, 8), dtype=torch.float64, device="cuda:0")
    raw, n_out, ass = ia.find_helices(ctx, hits, [0, ev.n_hits], sched, max_per_event=nh)
    torch.cuda.synchronize()
    n = int(n_out.cpu()[0])
    return ia.decode(raw, ia.HELIX_DTYPE)[:n], ass.cpu().numpy()[:ev.n_hits]


def test_serve_matches_solo_and_oracle():
    import torch
    assert torch.cuda.is_available()
    nh = KW["n_helix_max"]
    sched = ia.Schedule.make(H.LO, H.HI, **KW)
    events = [toymc.config_event(5, i) for i in range(48)]
    arrivals = serve.poisson_arrivals(len(events), rate=20000.0, seed=3)
    reqs = [serve.Request(i, ev.hits, float(t)) for i, (ev, t) in enumerate(zip(events, arrivals))]
    # small slots so that several batches of different sizes run concurrently
    per_event = ia.Context.scratch_needed(sched, 1000)
    loop = serve.ServeLoop(sched, max_per_event=nh, n_slots=3, scratch_budget=3 * 6 * per_event, max_batch=6)
    try:
        done = loop.run(reqs)
    finally:
        loop.close()
    assert sorted(r.rid for r in done) == list(range(len(events)))
    assert all(np.isfinite(r.done) and r.done >= r.arrival for r in done)
    ctx = ia.Context(0, scratch_bytes=per_event + (1 << 20))
    so = oracle.make_sched(H.LO, H.HI, **KW)
    try:
        for r in sorted(done, key=lambda r: r.rid):
            ev = events[r.rid]
            hel_1, ass_1 = _solo(ctx, ev, sched, nh)
            assert r.helices.tobytes() == hel_1.tobytes(), r.rid
            assert np.array_equal(r.assigned, ass_1), r.rid
            if r.rid % 8 == 0:
                ref, ref_ass = oracle.find_helices(ev.hits, so, max_out=nh)
                assert len(ref) == len(r.helices)
                for h in range(len(ref)):
                    assert np.array_equal(r.helices[h]["p"], ref[h]["p"])
                    assert np.array_equal(r.helices[h]["err"], ref[h]["err"])
                assert np.array_equal(r.assigned, ref_ass)
    finally:
        ctx.close()
    st = serve.latency_stats(done)
    assert st["p99_ms"] >= st["p50_ms"] > 0
