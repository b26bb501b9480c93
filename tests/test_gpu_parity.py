"""GPU parity: libia (HIP, gfx950) against the FP64 CPU oracle.

FP64 arithmetic on both sides follows the same IEEE operation sequence, so
votes, selections, estimates and helices must be identical bit for bit.
Inputs are seeded synthetic events; nothing here reads stored GPU output.
"""
import ctypes as C

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
    c = ia.Context(0, scratch_bytes=256 << 20)
    yield c
    c.close()


def _dev_hits(hits):
    torch = _torch()
    a = np.ascontiguousarray(hits).view(np.float64).reshape(-1, 8) if len(hits) else np.zeros((0, 8))
    return torch.from_numpy(a.copy()).to("cuda:0")


def _dev_boxes(boxes):
    torch = _torch()
    b = np.atleast_1d(boxes)
    a = np.concatenate([b["lo"], b["hi"]], axis=1).astype(np.float64)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _votes_np(t):
    return t.cpu().numpy().astype(np.uint16)


def _gpu_votes(ctx, hits, parents, split, active=None):
    torch = _torch()
    act = None if active is None else torch.from_numpy(np.asarray(active, np.uint8)).to("cuda:0")
    v = ia.vote_level(ctx, _dev_hits(hits), _dev_boxes(parents), split, active=act)
    torch.cuda.synchronize()
    return _votes_np(v)


@pytest.mark.parametrize("prefilter", [0, -1])
def test_level0_votes_bit_exact_cfg1(ctx, prefilter):
    """Single event, 12^5 level-0 grid (the plain FP64 single-level workload)."""
    ctx.set_prefilter(prefilter)
    for ev_i in range(2):
        ev = toymc.config_event(1, ev_i)
        print(f"cfg1 event {ev_i} N={ev.n_hits}", flush=True)
        root = oracle.make_box(H.LO, H.HI)
        ref = oracle.vote_level(ev.hits, root, [12] * 5)
        got = _gpu_votes(ctx, ev.hits, root, [12] * 5)
        assert got.shape == ref.shape
        bad = np.flatnonzero(got != ref)
        assert bad.size == 0, (bad[:10], got[bad[:10]], ref[bad[:10]])
    ctx.set_prefilter(-1)


def test_refinement_shape_votes_bit_exact(ctx):
    """32 parents split 4^5 (a refinement level) on a noisy event with bands."""
    ev = toymc.config_event(2, 3)
    root = oracle.make_box(H.LO, H.HI)
    v0 = oracle.vote_level(ev.hits, root, [8] * 5)
    idx, _ = oracle.topk(v0, 32)
    parents = np.array([oracle.box_child(root, [8] * 5, i) for i in idx])
    ref = oracle.vote_level(ev.hits, parents, [4] * 5)
    got = _gpu_votes(ctx, ev.hits, parents, [4] * 5)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("prefilter", [0, 1])
@pytest.mark.parametrize("tile", [64, 128, 256])
@pytest.mark.parametrize("split,n_par", [((3, 5, 2, 7, 3), 5), ((1, 1, 1, 1, 1), 300), ((2, 3, 1, 1, 1), 77),
                                         ((5, 1, 4, 1, 2), 3), ((4, 4, 4, 4, 4), 32)])
def test_ragged_shapes_bit_exact(ctx, split, n_par, tile, prefilter):
    """Shapes with ragged tiles (several triples per workgroup, partial last
    tile) under every vote-kernel tile (one box per lane, hits split over 2
    or 4 waves), with the (triple, hit) pre-filter off and forced on."""
    ctx.set_vote_tile(tile)
    ctx.set_prefilter(prefilter)
    ev = toymc.config_event(2, 5)
    rng = np.random.default_rng(41)
    t = ev.truth[0]
    w = (H.HI - H.LO) * 0.02
    parents = np.array([oracle.make_box(t - w * rng.uniform(0.2, 1, 5), t + w * rng.uniform(0.2, 1, 5))
                        for _ in range(n_par)])
    ref = oracle.vote_level(ev.hits, parents, split)
    try:
        got = _gpu_votes(ctx, ev.hits, parents, split)
    finally:
        ctx.set_vote_tile(0)
        ctx.set_prefilter(-1)
    assert np.array_equal(got, ref)


def test_far_boxes_take_the_plain_path_bit_exact(ctx):
    """Box centres far outside the physical (z0, tanl) range, where the
    correction eps of Eq. ApproxPhi exceeds pi/4 for many (box, hit) pairs:
    there the kernels' per-box evaluation leaves its branch-free form (whose
    sin/cos skip the range reduction) for the plain one.  Votes must still
    match the oracle bit for bit.  The host first checks, with the oracle's
    own intermediate values, that such pairs occur."""
    ev = toymc.config_event(2, 4)
    lo = np.array(H.LO, dtype=float)
    hi = np.array(H.HI, dtype=float)
    lo[3], hi[3], lo[4], hi[4] = -100.0, 100.0, -8.0, 8.0
    root = oracle.make_box(lo, hi)
    split = [5, 5, 5, 8, 8]
    pr = oracle.prep_hits(ev.hits)
    stereo = np.flatnonzero((pr["axial"] == 0) & (pr["valid"] == 1))
    rng = np.random.default_rng(7)
    i_eps = oracle.STEREO_DEBUG_NAMES.index("eps")
    n_big = 0
    for _ in range(200):
        c = lo + (hi - lo) * rng.random(5)
        for h in rng.choice(stereo, size=3, replace=False):
            ok, _, dbg = oracle.stereo_e(pr[h], c, 1, debug=True)
            n_big += np.isfinite(dbg[i_eps]) and abs(dbg[i_eps]) >= np.pi / 4
    assert n_big > 40, n_big
    ref = oracle.vote_level(ev.hits, root, split)
    got = _gpu_votes(ctx, ev.hits, root, split)
    assert np.array_equal(got, ref)


def test_edge_cases_hits(ctx):
    torch = _torch()
    root = oracle.make_box(H.LO, H.HI)
    # no hits
    got = _gpu_votes(ctx, np.zeros(0, dtype=toymc.HIT_DTYPE), root, [4] * 5)
    assert got.shape == (4 ** 5,) and not got.any()
    # malformed hits never vote and are counted
    ev = toymc.config_event(1, 9)
    hits = ev.hits.copy()
    bad = hits[:4].copy()
    bad[0]["drift"] = -1.0
    bad[1]["z1"] = bad[1]["z0"]
    bad[2]["x0"] = np.nan
    bad[3]["band"] = -1.0
    both = np.concatenate([hits, bad])
    ctx.clear_status()
    got = _gpu_votes(ctx, both, root, [6] * 5)
    ref = oracle.vote_level(hits, root, [6] * 5)
    assert np.array_equal(got, ref)
    flags, nbad = ctx.status()
    assert flags & 1 and nbad == 4
    ctx.clear_status()
    # active mask
    act = np.ones(ev.n_hits, np.uint8)
    act[::3] = 0
    got = _gpu_votes(ctx, hits, root, [6] * 5, active=act)
    ref = oracle.vote_level(hits, root, [6] * 5, active=act)
    assert np.array_equal(got, ref)
    # many hits (several chunks of the staging loop at level 0)
    ev5 = toymc.config_event(5, 3)
    many = np.concatenate([ev5.hits] * 4)[:700]
    parents = np.array([oracle.make_box(H.LO, H.HI)])
    got = _gpu_votes(ctx, many, parents, [3, 4, 3, 2, 2])
    ref = oracle.vote_level(many, parents, [3, 4, 3, 2, 2])
    assert np.array_equal(got, ref)
    del torch


@pytest.mark.parametrize("n,k,vmax", [(1, 1, 3), (7, 32, 2), (1000, 32, 3), (32768, 32, 20),
                                      (1048576, 32, 24), (250000, 64, 1), (5000, 4096, 9)])
def test_refine_topk_matches_oracle(ctx, n, k, vmax):
    torch = _torch()
    rng = np.random.default_rng(n + k)
    v = rng.integers(0, vmax + 1, n).astype(np.uint16)
    # one parent split n ways along d0: box index = child index
    root = oracle.make_box(H.LO, H.HI)
    parents = np.array([root])
    split = [n, 1, 1, 1, 1]
    sel, idx, sv = ia.refine(ctx, _dev_boxes(parents), split, torch.from_numpy(v).to("cuda:0"), vmax, k)
    torch.cuda.synchronize()
    ridx, rv = oracle.topk(v, k)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(sv.cpu().numpy().astype(np.uint16), rv)
    selb = sel.cpu().numpy()
    for r in range(min(len(ridx), 50)):
        b = oracle.box_child(root, split, ridx[r])
        assert np.array_equal(selb[r, :5], b["lo"]) and np.array_equal(selb[r, 5:], b["hi"])


def test_estimate_bit_exact(ctx):
    torch = _torch()
    ev = toymc.config_event(2, 4)
    root = oracle.make_box(H.LO, H.HI)
    v0 = oracle.vote_level(ev.hits, root, [8] * 5)
    idx, _ = oracle.topk(v0, 32)
    parents = np.array([oracle.box_child(root, [8] * 5, i) for i in idx])
    votes = oracle.vote_level(ev.hits, parents, [4] * 5)
    p, err, n = oracle.estimate(parents, [4] * 5, votes, votes.max())
    raw = ia.estimate(ctx, _dev_boxes(parents), [4] * 5, torch.from_numpy(votes).to("cuda:0"))
    got = ia.decode(raw, ia.ESTIMATE_DTYPE)[0]
    assert got["vmax"] == votes.max() and got["n_argmax"] == n
    assert np.array_equal(got["p"], p) and np.array_equal(got["err"], err)
    # level-0 estimate over a non-power-of-two grid
    v12 = oracle.vote_level(ev.hits, root, [12] * 5)
    p, err, n = oracle.estimate(np.array([root]), [12] * 5, v12, v12.max())
    raw = ia.estimate(ctx, _dev_boxes(root), [12] * 5, torch.from_numpy(v12).to("cuda:0"))
    got = ia.decode(raw, ia.ESTIMATE_DTYPE)[0]
    assert got["n_argmax"] == n and np.array_equal(got["p"], p) and np.array_equal(got["err"], err)


def _compare_find(ctx, events, sched_o, sched_g, max_out=4):
    torch = _torch()
    hits = np.concatenate([e.hits for e in events])
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])]).astype(np.int32)
    raw, n_out, assigned = ia.find_helices(ctx, _dev_hits(hits), off, sched_g, max_per_event=max_out)
    torch.cuda.synchronize()
    hel = ia.decode(raw, ia.HELIX_DTYPE).reshape(len(events), max_out)
    n_out = n_out.cpu().numpy()
    assigned = assigned.cpu().numpy()
    for e, ev in enumerate(events):
        ref, ref_ass = oracle.find_helices(ev.hits, sched_o, max_out=max_out)
        assert n_out[e] == len(ref), (e, n_out[e], len(ref))
        for h in range(len(ref)):
            g, r = hel[e, h], ref[h]
            assert np.array_equal(g["p"], r["p"]) and np.array_equal(g["err"], r["err"]), (e, h, g, r)
            assert (g["votes"], g["n_assigned"], g["n_argmax"]) == (r["votes"], r["n_assigned"], r["n_argmax"])
        assert np.array_equal(assigned[off[e]:off[e + 1]], ref_ass)


def test_find_helices_full_schedule_cfg2(ctx):
    """The measured workload: 16^5 grid, 4 levels of top-32 split 4^5, FP64."""
    events = [toymc.config_event(2, i) for i in range(2)]
    so = H.full_sched(oracle)
    sg = ia.Schedule.make(H.LO, H.HI, [16] * 5)
    _compare_find(ctx, events, so, sg, max_out=1)


def test_find_helices_multi_helix_small_grid(ctx):
    """Greedy multi-helix passes with hit removal (smaller grids for the oracle)."""
    events = [toymc.config_event(4, i) for i in range(3)]
    kw = dict(bins=[8] * 5, n_refine=2, top_k=16, split=[2] * 5, v_min=10, n_helix_max=4)
    so = oracle.make_sched(H.LO, H.HI, **kw)
    sg = ia.Schedule.make(H.LO, H.HI, **kw)
    _compare_find(ctx, events, so, sg, max_out=4)


def test_deterministic_repeat(ctx):
    ev = toymc.config_event(2, 6)
    root = oracle.make_box(H.LO, H.HI)
    a = _gpu_votes(ctx, ev.hits, root, [16] * 5)
    b = _gpu_votes(ctx, ev.hits, root, [16] * 5)
    assert np.array_equal(a, b)


def _run_gpu(ctx, events, sched, max_out):
    torch = _torch()
    hits = np.concatenate([e.hits for e in events]) if events else np.zeros(0, dtype=toymc.HIT_DTYPE)
    off = np.concatenate([[0], np.cumsum([e.n_hits for e in events])]).astype(np.int32)
    raw, n_out, assigned = ia.find_helices(ctx, _dev_hits(hits), off, sched, max_per_event=max_out)
    torch.cuda.synchronize()
    hel = ia.decode(raw, ia.HELIX_DTYPE).reshape(max(1, len(events)), max_out)
    return hel, n_out.cpu().numpy(), assigned.cpu().numpy(), off


def test_batch_mix_invariance(ctx):
    """Each event's result is the same alone, in one batch, and in small
    batches (uneven hit counts, multi-helix passes, full 16^5 schedule)."""
    events = [toymc.config_event(4, i) for i in range(10)]
    sched = ia.Schedule.make(H.LO, H.HI, [16] * 5, n_helix_max=5)
    hel_b, n_b, ass_b, off = _run_gpu(ctx, events, sched, 5)
    ctx.set_batch(3)
    try:
        hel_c, n_c, ass_c, _ = _run_gpu(ctx, events, sched, 5)
    finally:
        ctx.set_batch(65535)
    assert np.array_equal(n_b, n_c) and np.array_equal(ass_b, ass_c)
    assert hel_b.tobytes() == hel_c.tobytes()
    for e, ev in enumerate(events):
        hel_1, n_1, ass_1, _ = _run_gpu(ctx, [ev], sched, 5)
        assert n_1[0] == n_b[e]
        assert hel_1[0, :n_1[0]].tobytes() == hel_b[e, :n_b[e]].tobytes()
        assert np.array_equal(ass_1[:ev.n_hits], ass_b[off[e]:off[e + 1]])


def test_batch_edge_events(ctx):
    """Empty events, a one-hit event and a large event in one batch match the oracle."""
    big = toymc.config_event(5, 7)
    one = toymc.config_event(1, 3)
    one_hit = type(one)(hits=one.hits[:1], truth=one.truth, owner=one.owner[:1], layer=one.layer[:1],
                        wire=one.wire[:1], sigma=0.0)
    empty = type(one)(hits=one.hits[:0], truth=one.truth, owner=one.owner[:0], layer=one.layer[:0],
                      wire=one.wire[:0], sigma=0.0)
    events = [empty, one_hit, big, empty, toymc.config_event(2, 9)]
    kw = dict(bins=[6] * 5, n_refine=2, top_k=8, split=[2] * 5, v_min=10, n_helix_max=3)
    so = oracle.make_sched(H.LO, H.HI, **kw)
    sg = ia.Schedule.make(H.LO, H.HI, **kw)
    hel, n_out, ass, off = _run_gpu(ctx, events, sg, 3)
    for e, ev in enumerate(events):
        ref, ref_ass = oracle.find_helices(ev.hits, so, max_out=3)
        assert n_out[e] == len(ref)
        for h in range(len(ref)):
            assert np.array_equal(hel[e, h]["p"], ref[h]["p"]) and np.array_equal(hel[e, h]["err"], ref[h]["err"])
            assert hel[e, h]["n_assigned"] == ref[h]["n_assigned"]
        assert np.array_equal(ass[off[e]:off[e + 1]], ref_ass)


def test_pruning_does_not_change_helices(ctx):
    """find_helices with and without triple pruning: identical helices,
    votes, hit assignments (multi-helix events, full schedule)."""
    events = [toymc.config_event(4, i) for i in range(20, 26)]
    sched = ia.Schedule.make(H.LO, H.HI, [16] * 5, n_helix_max=5)
    hel_p, n_p, ass_p, _ = _run_gpu(ctx, events, sched, 5)
    ctx.set_pruning(False)
    try:
        hel_f, n_f, ass_f, _ = _run_gpu(ctx, events, sched, 5)
    finally:
        ctx.set_pruning(True)
    assert np.array_equal(n_p, n_f) and np.array_equal(ass_p, ass_f)
    for e in range(len(events)):
        assert hel_p[e, :n_p[e]].tobytes() == hel_f[e, :n_f[e]].tobytes()


def test_autotune_keeps_results(ctx):
    """The autotuner's tile table (one entry per level size, tiles of 64, 128
    or 256 boxes) does not change the search's results."""
    events = [toymc.config_event(4, i) for i in range(30, 36)]
    sched = ia.Schedule.make(H.LO, H.HI, [16] * 5, n_helix_max=5)
    hel_a, n_a, ass_a, off = _run_gpu(ctx, events, sched, 5)
    hits = _dev_hits(np.concatenate([e.hits for e in events]))
    table = ctx.autotune(hits, off, sched, max_per_event=5)
    assert set(table) == {16 ** 5, 32 * 4 ** 5} and set(table.values()) <= {64, 128, 256}
    hel_b, n_b, ass_b, _ = _run_gpu(ctx, events, sched, 5)
    assert np.array_equal(n_a, n_b) and np.array_equal(ass_a, ass_b)
    for e in range(len(events)):
        assert hel_a[e, :n_a[e]].tobytes() == hel_b[e, :n_b[e]].tobytes()


def test_parent_filter_does_not_change_results(ctx):
    """find_helices with and without the parent-level exclusion at the
    refinement levels: identical helices, votes and hit assignments, in FP64
    and in the mixed schedule."""
    events = [toymc.config_event(4, i) for i in range(40, 46)] + [toymc.config_event(5, i) for i in range(3)]
    for prec in (None, [ia.FP32] * 3 + [ia.FP64] * 2):
        sched = ia.Schedule.make(H.LO, H.HI, [16] * 5, n_helix_max=5, prec=prec)
        hel_a, n_a, ass_a, _ = _run_gpu(ctx, events, sched, 5)
        ctx.set_parent_filter(False)
        try:
            hel_b, n_b, ass_b, _ = _run_gpu(ctx, events, sched, 5)
        finally:
            ctx.set_parent_filter(True)
        assert np.array_equal(n_a, n_b) and np.array_equal(ass_a, ass_b)
        for e in range(len(events)):
            assert hel_a[e, :n_a[e]].tobytes() == hel_b[e, :n_b[e]].tobytes()


def test_classification_counters_and_timing(ctx):
    """The classification's work counters and the per-kernel timing record
    of one ia_vote_level call: one outer residual G per (triple, used hit),
    one axial test per axial pair (and an exact G for some of them), one set
    of pair magnitudes and one magnitude bound per stereo pair in the first
    stage; in the second, at most two enclosures and as many inclusion proofs
    per deferred pair; one timed launch each of the two stages and of the
    vote."""
    torch = _torch()
    ev = toymc.config_event(2, 3)
    prep = oracle.prep_hits(ev.hits)
    used = prep["valid"] == 1
    n_ax, n_st = int((used & (prep["axial"] == 1)).sum()), int((used & (prep["axial"] == 0)).sum())
    root = oracle.make_box(H.LO, H.HI)
    split = [9, 10, 11, 4, 4]
    n_tr = 9 * 10 * 11
    ctx.clear_status()
    ctx.profile_kernels()
    ctx.set_profiling(True)
    ctx.set_work_counting(True)
    try:
        v = ia.vote_level(ctx, _dev_hits(ev.hits), _dev_boxes(root), split)
        torch.cuda.synchronize()
    finally:
        ctx.set_profiling(False)
        ctx.set_work_counting(False)
    kp = ctx.profile_kernels()
    cw = ctx.classify_work()["fp64"]
    assert kp[("classify", "fp64")][0] == 1 and kp[("vote", "fp64")][0] == 1
    assert kp[("classify_defer", "fp64")][0] == 1
    assert kp[("classify", "fp32")][0] == 0 and kp[("classify", "fp64")][1] > 0
    assert cw["G"] == n_tr * (n_ax + n_st)
    assert cw["axial"] == n_tr * n_ax and 0 < cw["G_exact"] < cw["axial"]
    assert cw["pairq"] == n_tr * n_st
    assert cw["magnitudes"] == cw["pairq"]
    assert 0 < cw["deferred"] < cw["pairq"]
    assert cw["deferred"] <= cw["enclosures"] <= 2 * cw["deferred"] and cw["inclusions"] <= cw["enclosures"]
    assert np.array_equal(v.cpu().numpy().astype(np.uint16),
                          oracle.vote_level(ev.hits, root, split))
