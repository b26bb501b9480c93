"""GPU parity of the window schedule (Sec. 3.3 re-gridding from all max-vote
boxes, the moved reference point, the forward-hit test) against the oracle.

Both sides run the same FP64 operation sequences, so helices (p, err,
reference point, votes, max-vote set sizes, hit assignments) must agree bit
for bit.  Inputs are seeded synthetic events.
"""
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


def _dev_hits(hits):
    torch = _torch()
    a = np.ascontiguousarray(hits).view(np.float64).reshape(-1, 8) if len(hits) else np.zeros((0, 8))
    return torch.from_numpy(a.copy()).to("cuda:0")


def _run_gpu(ctx, events, sched, max_out):
    torch = _torch()
    hits = np.concatenate([e.hits for e in events]) if events else np.zeros(0, dtype=toymc.HIT_DTYPE)
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])]).astype(np.int32)
    raw, n_out, assigned = ia.find_helices(ctx, _dev_hits(hits), off, sched, max_per_event=max_out)
    torch.cuda.synchronize()
    hel = ia.decode(raw, ia.HELIX_DTYPE).reshape(max(1, len(events)), max_out)
    return hel, n_out.cpu().numpy(), assigned.cpu().numpy(), off


def _compare(ctx, events, kw, max_out, n_threads=0):
    so = oracle.make_sched(H.LO, H.HI, **kw)
    sg = ia.Schedule.make(H.LO, H.HI, **kw)
    hel, n_out, assigned, off = _run_gpu(ctx, events, sg, max_out)
    for e, ev in enumerate(events):
        ref, ref_ass = oracle.find_helices(ev.hits, so, max_out=max_out, n_threads=n_threads)
        assert n_out[e] == len(ref), (e, n_out[e], len(ref))
        for h in range(len(ref)):
            g, r = hel[e, h], ref[h]
            assert np.array_equal(g["p"], r["p"]), (e, h, g["p"], r["p"])
            assert np.array_equal(g["err"], r["err"]), (e, h, g["err"], r["err"])
            assert np.array_equal(g["ref"], r["ref"]), (e, h, g["ref"], r["ref"])
            assert (g["votes"], g["n_assigned"], g["n_argmax"]) == (r["votes"], r["n_assigned"], r["n_argmax"])
        assert np.array_equal(assigned[off[e]:off[e + 1]], ref_ass), e
    return hel, n_out


def _kw(**over):
    kw = dict(toymc.WINDOW_KW)
    kw.update(over)
    return kw


@pytest.mark.parametrize("cfg,wdrop,hitsel", [(3, 0, 0), (2, 0, 0), (2, 2, 1), (3, 1, 1)])
def test_window_schedule_matches_oracle(ctx, cfg, wdrop, hitsel):
    """The full window schedule (16^5, 16^5 window, move, four 12^5 windows) on
    two events: helices, errors, reference points and assignments bit-exact."""
    events = [toymc.config_event(cfg, i) for i in (0, 1)]
    hel, n_out = _compare(ctx, events, _kw(wdrop=wdrop, hitsel=hitsel), max_out=1)
    if cfg == 3:
        # noiseless: the search recovers the generated helix
        for e, ev in enumerate(events):
            assert toymc.recovered(hel[e, 0]["p"], ev.truth[0])


def test_window_multi_helix_full_schedule(ctx):
    """A multi-helix event (greedy passes with hit removal, each pass back in
    the origin's frame) under the full window schedule."""
    events = [toymc.config_event(4, 2)]
    _compare(ctx, events, _kw(n_helix_max=3, wdrop=1, hitsel=1), max_out=3)


def test_window_pruning_modes_agree(ctx):
    """Pruning off, by the largest lower bound, and with the probe pass (the
    default): identical helices and assignments on a batch of multi-helix
    events under the full window schedule, and the probe's threshold leaves
    fewer per-box evaluations."""
    events = [toymc.config_event(4, i) for i in range(30, 36)]
    sched = ia.Schedule.make(H.LO, H.HI, **_kw(n_helix_max=3, wdrop=1, hitsel=1))
    res, evals = {}, {}
    try:
        for mode in ("probe", "lower", "off"):
            ctx.set_pruning(mode != "off", probe=mode == "probe")
            ctx.clear_status()
            res[mode] = _run_gpu(ctx, events, sched, 3)
            evals[mode] = ctx.work()[0]
    finally:
        ctx.set_pruning(True)
    hel, n_out, assigned, _ = res["probe"]
    for mode in ("lower", "off"):
        h2, n2, a2, _ = res[mode]
        assert np.array_equal(n_out, n2) and np.array_equal(assigned, a2), mode
        for e in range(len(events)):
            assert hel[e, :n_out[e]].tobytes() == h2[e, :n2[e]].tobytes(), (mode, e)
    assert evals["probe"] < evals["lower"] < evals["off"], evals


def test_window_small_grids_batch_edges(ctx):
    """Empty events, a one-hit event and a large event next to ordinary ones in
    one batch (small window grids so that the oracle runs quickly)."""
    big = toymc.config_event(5, 7)
    one = toymc.config_event(1, 3)
    one_hit = type(one)(hits=one.hits[:1], truth=one.truth, owner=one.owner[:1], layer=one.layer[:1],
                        wire=one.wire[:1], sigma=0.0)
    empty = type(one)(hits=one.hits[:0], truth=one.truth, owner=one.owner[:0], layer=one.layer[:0],
                      wire=one.wire[:0], sigma=0.0)
    events = [empty, one_hit, big, empty, toymc.config_event(2, 9), toymc.config_event(4, 5)]
    for wdrop, hitsel in ((0, 0), (1, 1)):
        kw = _kw(bins=[6] * 5, n_refine=3, lbins=[[6] * 5, [6] * 5, [5] * 5, [5] * 5], n_helix_max=3, wdrop=wdrop,
                 hitsel=hitsel)
        _compare(ctx, events, kw, max_out=3)


@pytest.mark.parametrize("move_level,wdrop,hitsel,disk", [(-1, 0, 0, 0.0), (0, 2, 1, 5e-3), (2, 1, 1, 0.0),
                                                         (-1, 1, 1, 5e-3)])
def test_window_move_levels(ctx, move_level, wdrop, hitsel, disk):
    """No move, a move after level 0, a move late: forward-test levels and
    frames follow the schedule."""
    events = [toymc.config_event(2, 3), toymc.config_event(3, 4)]
    kw = _kw(bins=[8] * 5, n_refine=3, move_level=move_level, lbins=[[8] * 5, [8] * 5, [7] * 5, [7] * 5],
             wdrop=wdrop, hitsel=hitsel, disk=disk)
    _compare(ctx, events, kw, max_out=1)


def test_window_mixed_precision(ctx):
    """FP32 at levels 0-2 and FP64 after, under the window schedule."""
    events = [toymc.config_event(3, 5), toymc.config_event(2, 6)]
    _compare(ctx, events, _kw(prec=[1, 1, 1, 0, 0, 0]), max_out=1)


def test_topk_forward_matches_oracle(ctx):
    """The forward-hit test in the top-k schedule."""
    events = [toymc.config_event(2, i) for i in (2, 3)]
    for disk in (0.0, 5e-3):
        kw = dict(bins=[8] * 5, n_refine=2, top_k=16, split=[2] * 5, forward=True, disk=disk)
        _compare(ctx, events, kw, max_out=1)


@pytest.mark.parametrize("forward,ref,disk", [(1, (0.0, 0.0), 0.0), (0, (0.31, -0.42), 0.0),
                                              (1, (-0.2, 0.45), 0.0), (0, (0.31, -0.42), 5e-3),
                                              (1, (0.0, 0.0), 2e-3), (2, (0.31, -0.42), 5e-3),
                                              (2, (-0.2, 0.45), 0.0)])
def test_vote_level_frame_matches_oracle(ctx, forward, ref, disk):
    """ia_vote_level with the forward test, a moved reference point and the
    disk condition."""
    torch = _torch()
    ev = toymc.config_event(2, 4)
    lo, hi = H.LO.copy(), H.HI.copy()
    lo[0], hi[0] = -0.05, 0.05
    root = oracle.make_box(lo, hi)
    ctx.set_vote_frame(forward, ref, disk)
    try:
        b = np.atleast_1d(root)
        par = torch.from_numpy(np.concatenate([b["lo"], b["hi"]], axis=1).astype(np.float64)).to("cuda:0")
        v = ia.vote_level(ctx, _dev_hits(ev.hits), par, [12] * 5)
        torch.cuda.synchronize()
        got = v.cpu().numpy().astype(np.uint16)
    finally:
        ctx.set_vote_frame(False, (0.0, 0.0))
    want = oracle.vote_level(ev.hits, root, [12] * 5, forward=forward, ref=ref, disk=disk)
    assert np.array_equal(got, want)


def test_window_recovery_rates(ctx):
    """Recovery of the generated helices by the default window schedule on 400
    noiseless single-helix events (the GPU path equals the oracle bit for bit,
    so this is the schedule's rate): at least 95 % within the tolerances.
    Smeared events with noise hits and noiseless multi-helix events are
    reported, not required."""
    kw = dict(toymc.WINDOW_KW)
    sg = ia.Schedule.make(H.LO, H.HI, **kw)
    events = [toymc.config_event(3, i) for i in range(400)]
    hel, n_out, _, _ = _run_gpu(ctx, events, sg, 1)
    rec = sum(toymc.recovered(hel[e, 0]["p"], ev.truth[0]) for e, ev in enumerate(events) if n_out[e] > 0)
    print(f"noiseless single-helix recovery {rec}/400")
    assert rec >= 380
    events = [toymc.config_event(2, i) for i in range(200)]
    hel, n_out, _, _ = _run_gpu(ctx, events, sg, 1)
    rec = sum(toymc.recovered(hel[e, 0]["p"], ev.truth[0]) for e, ev in enumerate(events) if n_out[e] > 0)
    print(f"smeared single-helix recovery (20 % noise hits) {rec}/200")
