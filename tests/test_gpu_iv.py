"""GPU parity of the sound whole-box levels (IA_IV: d^Ax enclosed over the
whole box, Phi enclosed through Eq. CSAXtoPHI_a) against the oracle, bit for
bit: one vote level, and the window and top-k schedules with IV levels."""
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
    c = ia.Context(0, scratch_bytes=512 << 20)
    yield c
    c.close()


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a).view(np.float64).reshape(-1, 8).copy()).to("cuda:0")


@pytest.mark.parametrize("cfg,bins", [(2, [8] * 5), (1, [7] * 5)])
def test_vote_level_iv(ctx, cfg, bins):
    torch = _torch()
    ev = toymc.config_event(cfg, 3)
    root = oracle.make_box(H.LO, H.HI)
    b = np.atleast_1d(root)
    par = torch.from_numpy(np.concatenate([b["lo"], b["hi"]], axis=1).astype(np.float64)).to("cuda:0")
    v = ia.vote_level(ctx, _dev(ev.hits), par, bins, prec=ia.IV)
    torch.cuda.synchronize()
    want = oracle.vote_level(ev.hits, root, bins, prec=oracle.IV)
    assert np.array_equal(v.cpu().numpy().astype(np.uint16), want)


def _compare(ctx, events, kw, max_out):
    torch = _torch()
    so = oracle.make_sched(H.LO, H.HI, **kw)
    sg = ia.Schedule.make(H.LO, H.HI, **kw)
    hits = np.concatenate([e.hits for e in events])
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])]).astype(np.int32)
    raw, n_out, ass = ia.find_helices(ctx, _dev(hits), off, sg, max_per_event=max_out)
    torch.cuda.synchronize()
    hel = ia.decode(raw, ia.HELIX_DTYPE).reshape(len(events), max_out)
    n_out, ass = n_out.cpu().numpy(), ass.cpu().numpy()
    for e, ev in enumerate(events):
        ref, ref_ass = oracle.find_helices(ev.hits, so, max_out=max_out)
        assert n_out[e] == len(ref), (e, n_out[e], len(ref))
        for h in range(len(ref)):
            g, r = hel[e, h], ref[h]
            assert np.array_equal(g["p"], r["p"]) and np.array_equal(g["err"], r["err"]), (e, h)
            assert np.array_equal(g["ref"], r["ref"])
            assert (g["votes"], g["n_assigned"], g["n_argmax"]) == (r["votes"], r["n_assigned"], r["n_argmax"])
        assert np.array_equal(ass[off[e]:off[e + 1]], ref_ass), e
    return hel, n_out


@pytest.mark.parametrize("prec,cfgs", [([ia.IV] * 4, ((2, 5), (3, 6))),
                                       ([ia.FP64, ia.FP64, ia.IV, ia.IV], ((2, 5), (3, 6), (4, 7)))])
def test_window_schedule_iv(ctx, prec, cfgs):
    events = [toymc.config_event(c, i) for c, i in cfgs]
    kw = dict(toymc.WINDOW_KW)
    kw.update(bins=[8] * 5, n_refine=3, lbins=[[8] * 5, [8] * 5, [7] * 5, [7] * 5], prec=prec, n_helix_max=2)
    _compare(ctx, events, kw, max_out=2)


def test_topk_schedule_iv(ctx):
    events = [toymc.config_event(2, i) for i in (8, 9)]
    kw = dict(bins=[8] * 5, n_refine=2, top_k=16, split=[2] * 5, forward=True, prec=[ia.FP64, ia.IV, ia.IV])
    _compare(ctx, events, kw, max_out=1)


def test_window_schedule_iv_full_size(ctx):
    """The default window schedule (16^5, 16^5, six 12^5 windows) with its
    last level IV, on a noiseless event: bit-exact and recovered."""
    events = [toymc.config_event(3, 10)]
    kw = dict(toymc.WINDOW_KW)
    kw["prec"] = [ia.FP64] * 7 + [ia.IV]
    hel, n_out = _compare(ctx, events, kw, max_out=1)
    assert n_out[0] == 1 and toymc.recovered(hel[0, 0]["p"], events[0].truth[0])
