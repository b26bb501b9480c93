"""The search captured once in a HIP graph (ia_find_helices_dev) and replayed
on new events: every replay equals the eager search of the same events, bit
for bit, with eager work and synchronisations between the replays."""
import numpy as np
import pytest

import paper_2401_04576_amd as ia
from paper_2401_04576_amd import toymc
from tests import _helpers as H

pytestmark = pytest.mark.gpu

E, MAX_HITS, NH = 12, 200, 5


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _eager(ctx, events, sched):
    torch = _torch()
    hits = np.concatenate([e.hits for e in events])
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])]).astype(np.int32)
    d = torch.from_numpy(hits.view(np.float64).reshape(-1, 8).copy()).to("cuda:0")
    raw, n_out, ass = ia.find_helices(ctx, d, off, sched, max_per_event=NH)
    torch.cuda.synchronize()
    return ia.decode(raw, ia.HELIX_DTYPE).reshape(len(events), NH), n_out.cpu().numpy(), ass.cpu().numpy()


def test_graph_replays_match_eager():
    torch = _torch()
    dev = torch.device("cuda:0")
    sched = ia.Schedule.make(H.LO, H.HI, [16] * 5, n_helix_max=NH)
    sets = [[toymc.config_event(4, 100 * k + i) for i in range(E)] for k in range(3)]
    for evs in sets:
        assert max(e.n_hits for e in evs) <= MAX_HITS
    ctx_g = ia.Context(0, scratch_bytes=512 << 20)
    ctx_e = ia.Context(0, scratch_bytes=256 << 20)
    hits_buf = torch.zeros((E * MAX_HITS, 8), dtype=torch.float64, device=dev)
    off_buf = torch.zeros(E + 1, dtype=torch.int32, device=dev)
    out = torch.zeros(E * NH * ia.HELIX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    n_out = torch.zeros(E, dtype=torch.int32, device=dev)
    assigned = torch.full((E * MAX_HITS,), -1, dtype=torch.int32, device=dev)

    def load(evs):
        h = np.concatenate([e.hits for e in evs])
        off = np.concatenate([[0], np.cumsum([e.n_hits for e in evs])]).astype(np.int32)
        hits_buf.zero_()
        hits_buf[:h.shape[0]].copy_(torch.from_numpy(h.view(np.float64).reshape(-1, 8).copy()))
        off_buf.copy_(torch.from_numpy(off))
        return off

    try:
        load(sets[0])
        ia.find_helices_dev(ctx_g, hits_buf, off_buf, MAX_HITS, sched, out, n_out, assigned, max_per_event=NH)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        with torch.cuda.graph(g, stream=s):
            ia.find_helices_dev(ctx_g, hits_buf, off_buf, MAX_HITS, sched, out, n_out, assigned,
                                max_per_event=NH, stream=s)
        for evs in sets + [sets[0]]:
            off = load(evs)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = ia.decode(out, ia.HELIX_DTYPE).reshape(E, NH)
            got_n = n_out.cpu().numpy()
            got_a = assigned.cpu().numpy()
            _ = (torch.ones(1000, device=dev) * 2).sum().item()      # eager work between replays
            ref, ref_n, ref_a = _eager(ctx_e, evs, sched)
            assert np.array_equal(got_n, ref_n)
            for e in range(E):
                assert got[e, :ref_n[e]].tobytes() == ref[e, :ref_n[e]].tobytes(), e
            assert np.array_equal(got_a[:off[-1]], ref_a)
        assert ctx_g.status()[0] & 4 == 0
    finally:
        ctx_g.close()
        ctx_e.close()


def test_dev_offsets_out_of_bounds_flagged():
    """An event larger than max_hits is not searched and sets status bit 2;
    the other events of the call are searched as in the host-offset search."""
    torch = _torch()
    dev = torch.device("cuda:0")
    sched = ia.Schedule.make(H.LO, H.HI, [8] * 5, n_refine=2, top_k=16, split=[2] * 5, n_helix_max=2)
    evs = [toymc.config_event(2, i) for i in range(3)]
    h = np.concatenate([e.hits for e in evs])
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in evs])]).astype(np.int32)
    max_hits = max(evs[0].n_hits, evs[1].n_hits)
    bad_off = off.copy()
    bad_off[3] = bad_off[2] + max_hits + 5              # the third event claims more than max_hits
    ctx = ia.Context(0, scratch_bytes=256 << 20)
    try:
        hits_buf = torch.zeros((int(bad_off[3]), 8), dtype=torch.float64, device=dev)
        hits_buf[:h.shape[0]].copy_(torch.from_numpy(h.view(np.float64).reshape(-1, 8).copy()))
        d_off = torch.from_numpy(bad_off).to(dev)
        out = torch.zeros(3 * 2 * ia.HELIX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        n_out = torch.zeros(3, dtype=torch.int32, device=dev)
        ctx.clear_status()
        ia.find_helices_dev(ctx, hits_buf, d_off, max_hits, sched, out, n_out, None, max_per_event=2)
        torch.cuda.synchronize()
        flags, _ = ctx.status()
        assert flags & 4
        got = ia.decode(out, ia.HELIX_DTYPE).reshape(3, 2)
        got_n = n_out.cpu().numpy()
        assert got_n[2] == 0
        raw, n1, _ = ia.find_helices(ctx, hits_buf[:off[2]], off[:3], sched, max_per_event=2)
        torch.cuda.synchronize()
        ref = ia.decode(raw, ia.HELIX_DTYPE).reshape(2, 2)
        ref_n = n1.cpu().numpy()
        assert np.array_equal(got_n[:2], ref_n)
        for e in range(2):
            assert got[e, :ref_n[e]].tobytes() == ref[e, :ref_n[e]].tobytes()
    finally:
        ctx.close()
