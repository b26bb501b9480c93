"""GPU parity at FP32 levels: libia's FP32 votes against the oracle's FP32
definition (bit for bit: the FP32 operation sequence is the same on both
sides), FP32 votes containing FP64 votes on the device, and the mixed
schedule (FP32 coarse levels, FP64 fine levels and fit) against the oracle
run with the same schedule."""
import numpy as np
import pytest

import oracle
import paper_2401_04576_amd as ia
from paper_2401_04576_amd import toymc
from tests import _helpers as H

pytestmark = pytest.mark.gpu

SLACK = 1e-6


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def ctx():
    _torch()
    c = ia.Context(0, scratch_bytes=256 << 20)
    c.set_fp32_slack(SLACK)
    yield c
    c.close()


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _dev_hits(hits):
    return _dev(np.ascontiguousarray(hits).view(np.float64).reshape(-1, 8).copy())


def _dev_boxes(boxes):
    b = np.atleast_1d(boxes)
    return _dev(np.concatenate([b["lo"], b["hi"]], axis=1).astype(np.float64))


def _votes(ctx, hits, parents, split, prec):
    torch = _torch()
    v = ia.vote_level(ctx, _dev_hits(hits), _dev_boxes(parents), split, prec=prec)
    torch.cuda.synchronize()
    return v.cpu().numpy().astype(np.uint16)


@pytest.mark.parametrize("prefilter", [0, -1])
@pytest.mark.parametrize("cfg,ev_i", [(1, 0), (2, 1), (5, 3)])
def test_fp32_level0_bit_exact(ctx, prefilter, cfg, ev_i):
    ev = toymc.config_event(cfg, ev_i)
    root = oracle.make_box(H.LO, H.HI)
    ref = oracle.vote_level(ev.hits, root, [12] * 5, prec=oracle.FP32, slack=SLACK)
    ctx.set_prefilter(prefilter)
    try:
        got = _votes(ctx, ev.hits, root, [12] * 5, ia.FP32)
    finally:
        ctx.set_prefilter(-1)
    assert np.array_equal(got, ref), np.flatnonzero(got != ref)[:10]
    v64 = _votes(ctx, ev.hits, root, [12] * 5, ia.FP64)
    assert (got.astype(np.int64) - v64).min() >= 0


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_fp32_refinement_shapes(ctx, tile):
    ev = toymc.config_event(2, 4)
    root = oracle.make_box(H.LO, H.HI)
    v0 = oracle.vote_level(ev.hits, root, [10] * 5, prec=oracle.FP32, slack=SLACK)
    top = np.argsort(-v0.astype(np.int64), kind="stable")[:13]
    parents = np.array([oracle.box_child(root, [10] * 5, int(b)) for b in top])
    split = [3, 4, 2, 5, 3]
    ref = oracle.vote_level(ev.hits, parents, split, prec=oracle.FP32, slack=SLACK)
    ctx.set_vote_tile(tile)
    try:
        got = _votes(ctx, ev.hits, parents, split, ia.FP32)
    finally:
        ctx.set_vote_tile(0)
    assert np.array_equal(got, ref)


def test_fp32_domain_edge_kappa_zero(ctx):
    """A grid whose kappa centres include 0 (radius beyond the FP32 domain):
    those stereo pairs vote, on both sides."""
    ev = toymc.config_event(1, 2)
    lo, hi = H.LO.copy(), H.HI.copy()
    lo[2], hi[2] = -0.3, 0.3
    root = oracle.make_box(lo, hi)
    split = [6, 6, 5, 6, 6]                       # odd kappa split: a centre at 0
    ref = oracle.vote_level(ev.hits, root, split, prec=oracle.FP32, slack=SLACK)
    got = _votes(ctx, ev.hits, root, split, ia.FP32)
    assert np.array_equal(got, ref)


def test_mixed_schedule_find_helices(ctx):
    """FP32 at levels 0-2, FP64 at 3-4 and in the fit: helices, votes and hit
    assignment equal the oracle's under the same schedule."""
    torch = _torch()
    kw = dict(bins=[10] * 5, n_refine=4, top_k=16, split=[3] * 5, v_min=10, n_helix_max=3)
    prec = [ia.FP32] * 3 + [ia.FP64] * 2
    so = oracle.make_sched(H.LO, H.HI, prec=prec, fp32_slack=SLACK, **kw)
    sg = ia.Schedule.make(H.LO, H.HI, prec=prec, fp32_slack=SLACK, **kw)
    events = [toymc.config_event(3, i) for i in range(3)] + [toymc.config_event(4, 5)]
    hits = np.concatenate([e.hits for e in events])
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])])
    raw, n_out, ass = ia.find_helices(ctx, _dev_hits(hits), off, sg, max_per_event=3)
    torch.cuda.synchronize()
    hel = ia.decode(raw, ia.HELIX_DTYPE).reshape(len(events), 3)
    n_out = n_out.cpu().numpy()
    ass = ass.cpu().numpy()
    for e, ev in enumerate(events):
        ref, ref_ass = oracle.find_helices(ev.hits, so, max_out=3)
        assert n_out[e] == len(ref)
        for h in range(len(ref)):
            assert np.array_equal(hel[e, h]["p"], ref[h]["p"])
            assert np.array_equal(hel[e, h]["err"], ref[h]["err"])
            assert int(hel[e, h]["votes"]) == int(ref[h]["votes"])
        assert np.array_equal(ass[off[e]:off[e + 1]], ref_ass)
