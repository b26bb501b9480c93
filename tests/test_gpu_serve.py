"""Serving over resident pools: continuous batching at helix-pass
granularity gives every event the result it gets alone, and that result
matches the oracle.

Events of the serving mix (1-10 helices, lognormal hit counts, 0-40 % noise)
arrive as a Poisson stream fast enough that the few rows of each pool are
refilled while other rows are still searching.
"""
import numpy as np
import pytest

import oracle
import paper_2401_04576_amd as ia
from paper_2401_04576_amd import serve, toymc
from tests import _helpers as H

pytestmark = pytest.mark.gpu


def _window_kw(**over):
    kw = dict(toymc.WINDOW_KW)
    kw.update(over)
    return kw


SMALL = _window_kw(bins=[6] * 5, n_refine=3, lbins=[[6] * 5, [6] * 5, [5] * 5, [5] * 5], v_min=10, n_helix_max=4)


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _solo(ctx, ev, sched, nh):
    torch = _torch()
    hits = torch.from_numpy(np.ascontiguousarray(ev.hits).view(np.float64).reshape(-1, 8).copy()).to("cuda:0") \
        if ev.n_hits else torch.zeros((0, 8), dtype=torch.float64, device="cuda:0")
    raw, n_out, ass = ia.find_helices(ctx, hits, [0, ev.n_hits], sched, max_per_event=nh)
    torch.cuda.synchronize()
    n = int(n_out.cpu()[0])
    return ia.decode(raw, ia.HELIX_DTYPE)[:n], ass.cpu().numpy()[:ev.n_hits]


def _same_as_oracle(r, ev, so, nh):
    ref, ref_ass = oracle.find_helices(ev.hits, so, max_out=nh)
    assert len(ref) == len(r.helices), (r.rid, len(ref), len(r.helices))
    for h in range(len(ref)):
        g = r.helices[h]
        assert np.array_equal(g["p"], ref[h]["p"]) and np.array_equal(g["err"], ref[h]["err"]), (r.rid, h)
        assert np.array_equal(g["ref"], ref[h]["ref"])
        assert (g["votes"], g["n_assigned"]) == (ref[h]["votes"], ref[h]["n_assigned"])
    assert np.array_equal(r.assigned, ref_ass), r.rid


def test_pool_serving_matches_solo_and_oracle():
    torch = _torch()
    nh = SMALL["n_helix_max"]
    sched = ia.Schedule.make(H.LO, H.HI, **SMALL)
    events = [toymc.config_event(5, i) for i in range(48)]
    arrivals = serve.poisson_arrivals(len(events), rate=20000.0, seed=3)
    reqs = [serve.Request(i, ev.hits, float(t)) for i, (ev, t) in enumerate(zip(events, arrivals))]
    # three small pools (a few rows each): rows are refilled while others search
    loop = serve.ServeLoop(sched, max_per_event=nh, scratch_budget=3 << 30, classes={128: 1, 256: 1, 1024: 1},
                           rows_cap=4)
    try:
        caps = loop.capacity()
        assert all(1 <= v <= 4 for v in caps.values()), caps
        done = loop.run(reqs)
    finally:
        loop.close()
    assert sorted(r.rid for r in done) == list(range(len(events)))
    assert all(np.isfinite(r.done) and r.done >= r.arrival for r in done)
    ctx = ia.Context(0, scratch_bytes=ia.Context.scratch_needed(sched, 1000) + (1 << 20))
    so = oracle.make_sched(H.LO, H.HI, **SMALL)
    try:
        for r in sorted(done, key=lambda r: r.rid):
            ev = events[r.rid]
            hel_1, ass_1 = _solo(ctx, ev, sched, nh)
            assert r.helices.tobytes() == hel_1.tobytes(), r.rid
            assert np.array_equal(r.assigned, ass_1), r.rid
            if r.rid % 8 == 0:
                _same_as_oracle(r, ev, so, nh)
    finally:
        ctx.close()
    st = serve.latency_stats(done)
    assert st["p99_ms"] >= st["p50_ms"] > 0
    torch.cuda.synchronize()


def test_pool_rows_are_reused_and_abandoned_rows_restart():
    """The pool API directly: a row admitted while another is mid-search, a
    row re-admitted after it finished, and a row abandoned mid-search and
    re-admitted with a new event all give the solo results."""
    torch = _torch()
    nh = SMALL["n_helix_max"]
    sched = ia.Schedule.make(H.LO, H.HI, **SMALL)
    ctx = ia.Context(0, scratch_bytes=1 << 30)
    evs = [toymc.config_event(4, 400 + i) for i in range(4)]

    def dev(e):
        return torch.from_numpy(np.ascontiguousarray(e.hits).view(np.float64).reshape(-1, 8).copy()).to("cuda:0")

    try:
        pool = ia.Pool(ctx, 2, 256, sched, max_per_event=nh)
        pool.admit([0], dev(evs[0]), [0, evs[0].n_hits])
        pool.step()
        pool.admit([1], dev(evs[1]), [0, evs[1].n_hits])        # row 0 is mid-search
        got = {}
        for _ in range(2 * nh + 2):
            pool.step()
            done, n_out = pool.poll()
            for r, ev_i in ((0, 0), (1, 1)):
                if done[r] and ev_i not in got:
                    got[ev_i] = pool.take(r, int(n_out[r]), evs[ev_i].n_hits)
        assert set(got) == {0, 1}
        pool.admit([0], dev(evs[2]), [0, evs[2].n_hits])        # reuse a finished row
        pool.step()
        pool.admit([0], dev(evs[3]), [0, evs[3].n_hits])        # abandon it mid-search
        for _ in range(nh + 1):
            pool.step()
        done, n_out = pool.poll()
        assert done[0]
        got[3] = pool.take(0, int(n_out[0]), evs[3].n_hits)
        with pytest.raises(ia.IAError):
            ia.find_helices(ctx, dev(evs[0]), [0, evs[0].n_hits], sched, max_per_event=nh)
        pool.close()
        for ev_i in (0, 1, 3):
            hel_1, ass_1 = _solo(ctx, evs[ev_i], sched, nh)
            assert got[ev_i][0].tobytes() == hel_1.tobytes(), ev_i
            assert np.array_equal(got[ev_i][1], ass_1), ev_i
    finally:
        ctx.close()


def test_pool_full_schedule_config5_event_matches_oracle():
    """A config-5 event (56 hits, 4 helices) under the full window schedule
    through the serving loop, against the oracle bit for bit."""
    nh = 3
    kw = _window_kw(n_helix_max=nh)
    sched = ia.Schedule.make(H.LO, H.HI, **kw)
    ev = toymc.config_event(5, 7)
    loop = serve.ServeLoop(sched, max_per_event=nh, scratch_budget=4 << 30, classes={128: 1}, rows_cap=2)
    try:
        done = loop.run([serve.Request(0, ev.hits, 0.0)])
    finally:
        loop.close()
    assert len(done) == 1
    _same_as_oracle(done[0], ev, oracle.make_sched(H.LO, H.HI, **kw), nh)
