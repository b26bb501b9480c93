"""GPU parity in the measured shapes and on the branches the smaller tests do
not reach: a full 16^5 level of ia_vote_level, an event of more than 1023
hits (the vote histogram in global memory), config-4 events under the full
top-k schedule with 5 helix passes, and a captured graph of the window
schedule replayed on new events, each against the oracle."""
import numpy as np
import pytest

import oracle
import paper_2401_04576_amd as ia
from paper_2401_04576_amd import toymc
from tests import _helpers as H

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def ctx():
    _torch()
    c = ia.Context(0, scratch_bytes=1 << 30)
    yield c
    c.close()


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a).view(np.float64).reshape(-1, 8).copy()).to("cuda:0")


def _find(ctx, events, sched, nh):
    torch = _torch()
    hits = np.concatenate([e.hits for e in events])
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])]).astype(np.int32)
    raw, n_out, ass = ia.find_helices(ctx, _dev(hits), off, sched, max_per_event=nh)
    torch.cuda.synchronize()
    return ia.decode(raw, ia.HELIX_DTYPE).reshape(len(events), nh), n_out.cpu().numpy(), ass.cpu().numpy(), off


def _check(events, hel, n_out, ass, off, so, nh):
    for e, ev in enumerate(events):
        ref, ref_ass = oracle.find_helices(ev.hits, so, max_out=nh)
        assert n_out[e] == len(ref), (e, n_out[e], len(ref))
        for h in range(len(ref)):
            g, r = hel[e, h], ref[h]
            assert np.array_equal(g["p"], r["p"]) and np.array_equal(g["err"], r["err"]), (e, h)
            assert np.array_equal(g["ref"], r["ref"])
            assert (g["votes"], g["n_assigned"], g["n_argmax"]) == (r["votes"], r["n_assigned"], r["n_argmax"])
        assert np.array_equal(ass[off[e]:off[e + 1]], ref_ass), e


def test_vote_level_full_16_grid_cfg2(ctx):
    """ia_vote_level over the 16^5 level-0 grid of a config-2 event."""
    torch = _torch()
    ev = toymc.config_event(2, 11)
    root = oracle.make_box(H.LO, H.HI)
    b = np.atleast_1d(root)
    par = torch.from_numpy(np.concatenate([b["lo"], b["hi"]], axis=1).astype(np.float64)).to("cuda:0")
    v = ia.vote_level(ctx, _dev(ev.hits), par, [16] * 5)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy().astype(np.uint16), oracle.vote_level(ev.hits, root, [16] * 5))


def _big_event(n_hits, seed):
    rng = toymc.rng_for(77, seed)
    return toymc.make_event(rng, n_helix=8, sigma=150e-6, noise_frac=0.4, n_hits=n_hits)


@pytest.mark.parametrize("mode", ["topk", "window"])
def test_event_above_1023_hits(ctx, mode):
    """An event of 1100 hits (vote histograms beyond the LDS bins) beside a
    small one, small grids, two helix passes."""
    big = _big_event(1100, 1)
    assert big.n_hits > 1023
    events = [big, toymc.config_event(2, 5)]
    if mode == "topk":
        kw = dict(bins=[6] * 5, n_refine=2, top_k=8, split=[2] * 5, v_min=10, n_helix_max=2)
    else:
        kw = dict(toymc.WINDOW_KW)
        kw.update(bins=[6] * 5, n_refine=3, lbins=[[6] * 5, [6] * 5, [5] * 5, [5] * 5], v_min=10, n_helix_max=2)
    so = oracle.make_sched(H.LO, H.HI, **kw)
    sg = ia.Schedule.make(H.LO, H.HI, **kw)
    hel, n_out, ass, off = _find(ctx, events, sg, 2)
    _check(events, hel, n_out, ass, off, so, 2)


def test_config4_full_topk_schedule_five_passes(ctx):
    """Two config-4 events under the literal schedule (16^5, four levels of the
    top 32 boxes split 4^5) with up to 5 greedy helix passes."""
    events = [toymc.config_event(4, i) for i in (3, 4)]
    kw = dict(toymc.TOPK_KW, v_min=10, n_helix_max=5)
    so = oracle.make_sched(H.LO, H.HI, **kw)
    sg = ia.Schedule.make(H.LO, H.HI, **kw)
    hel, n_out, ass, off = _find(ctx, events, sg, 5)
    _check(events, hel, n_out, ass, off, so, 5)


def test_window_graph_replays_match_oracle():
    """ia_find_helices_dev under the window schedule, captured once and replayed
    on two new sets of events (eager work and synchronisations between the
    replays): every replay equals the oracle."""
    torch = _torch()
    dev = torch.device("cuda:0")
    E, MAXH, NH = 4, 200, 3
    kw = dict(toymc.WINDOW_KW)
    kw.update(bins=[8] * 5, n_refine=3, lbins=[[8] * 5, [8] * 5, [7] * 5, [7] * 5], v_min=10, n_helix_max=NH)
    so = oracle.make_sched(H.LO, H.HI, **kw)
    sg = ia.Schedule.make(H.LO, H.HI, **kw)
    sets = [[toymc.config_event(4, 300 + 10 * k + i) for i in range(E)] for k in range(3)]
    ctx = ia.Context(0, scratch_bytes=1 << 30)
    hits_buf = torch.zeros((E * MAXH, 8), dtype=torch.float64, device=dev)
    off_buf = torch.zeros(E + 1, dtype=torch.int32, device=dev)
    out = torch.zeros(E * NH * ia.HELIX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    n_out = torch.zeros(E, dtype=torch.int32, device=dev)
    assigned = torch.full((E * MAXH,), -1, dtype=torch.int32, device=dev)

    def load(evs):
        h = np.concatenate([e.hits for e in evs])
        off = np.concatenate([[0], np.cumsum([e.n_hits for e in evs])]).astype(np.int32)
        hits_buf.zero_()
        hits_buf[:h.shape[0]].copy_(torch.from_numpy(h.view(np.float64).reshape(-1, 8).copy()))
        off_buf.copy_(torch.from_numpy(off))
        return off

    try:
        load(sets[0])
        ia.find_helices_dev(ctx, hits_buf, off_buf, MAXH, sg, out, n_out, assigned, max_per_event=NH)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        with torch.cuda.graph(g, stream=s):
            ia.find_helices_dev(ctx, hits_buf, off_buf, MAXH, sg, out, n_out, assigned, max_per_event=NH,
                                stream=s)
        torch.cuda.synchronize()
        for evs in sets[1:]:
            off = load(evs)
            assigned.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            _ = torch.ones(1000, device=dev).sum().item()   # eager work between the replays
            hel = ia.decode(out, ia.HELIX_DTYPE).reshape(E, NH)
            _check(evs, hel, n_out.cpu().numpy(), assigned.cpu().numpy(), off, so, NH)
    finally:
        ctx.close()
