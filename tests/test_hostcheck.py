"""The HIP library's vote arithmetic, compiled for the CPU (tests/hostcheck),
against the oracle: identical votes with and without the (triple, hit)
pre-filter, whose classes skip the per-box evaluation of pairs proved to
vote nowhere or everywhere in a triple.  A missed or extra vote would show
a class proof is unsound."""
import numpy as np
import pytest

from paper_2401_04576_amd import toymc
from tests import _helpers as H
from tests import hostcheck


@pytest.mark.parametrize("cfg,ev_i", [(1, 0), (2, 1), (2, 2), (5, 4)])
def test_device_arithmetic_matches_oracle_level0(orc, cfg, ev_i):
    ev = toymc.config_event(cfg, ev_i)
    root = orc.make_box(H.LO, H.HI)
    ref = orc.vote_level(ev.hits, root, [10] * 5)
    for filt in (False, True):
        got, stats = hostcheck.vote_level(ev.hits, root, [10] * 5, filt)
        assert np.array_equal(got, ref), (filt, np.flatnonzero(got != ref)[:10])


def test_prefilter_sound_on_refinement_shapes(orc):
    rng = np.random.default_rng(51)
    for ev_i in range(3):
        ev = toymc.config_event(2, 10 + ev_i)
        t = ev.truth[0]
        w = (H.HI - H.LO) * np.array([0.05, 0.02, 0.05, 0.3, 0.3])
        parents = np.array([orc.make_box(t - w * rng.uniform(0.1, 1, 5), t + w * rng.uniform(0.1, 1, 5))
                            for _ in range(6)])
        ref = orc.vote_level(ev.hits, parents, [3, 3, 3, 8, 8])
        got, stats = hostcheck.vote_level(ev.hits, parents, [3, 3, 3, 8, 8], True)
        assert np.array_equal(got, ref)


def test_prefilter_effect_level0():
    """Fraction of stereo (triple, hit) pairs the pre-filter removes on the
    16^5 level-0 grid of the measured workload (ideal: 83 %)."""
    ev = toymc.config_event(2, 0)
    root = np.zeros(1, dtype=[("lo", "f8", (5,)), ("hi", "f8", (5,))])
    root["lo"], root["hi"] = H.LO, H.HI
    v_on, s_on = hostcheck.vote_level(ev.hits, root, [16] * 5, True)
    v_off, s_off = hostcheck.vote_level(ev.hits, root, [16] * 5, False)
    assert np.array_equal(v_on, v_off)
    frac = s_on[1] / s_on[0]
    print(f"pre-filter removes {frac:.1%} of stereo (triple, hit) pairs; "
          f"stereo box evaluations {s_on[2]} vs {s_off[2]}")
    assert frac > 0.3


SLACK = 1e-6


@pytest.mark.parametrize("cfg,ev_i", [(1, 1), (2, 0), (5, 4)])
def test_device_fp32_arithmetic_matches_oracle(orc, cfg, ev_i):
    """The library's FP32 vote arithmetic (CPU build) equals the oracle's FP32
    votes on a level-0 grid and a refinement level, pre-filter on and off."""
    ev = toymc.config_event(cfg, ev_i)
    root = orc.make_box(H.LO, H.HI)
    ref = orc.vote_level(ev.hits, root, [10] * 5, prec=orc.FP32, slack=SLACK)
    for filt in (False, True):
        got, _ = hostcheck.vote_level(ev.hits, root, [10] * 5, filt, f32=True, slack=SLACK)
        assert np.array_equal(got, ref), (filt, np.flatnonzero(got != ref)[:10])
    top = np.argsort(-ref.astype(np.int64), kind="stable")[:6]
    parents = np.array([orc.box_child(root, [10] * 5, int(b)) for b in top])
    ref1 = orc.vote_level(ev.hits, parents, [4] * 5, prec=orc.FP32, slack=SLACK)
    got1, stats = hostcheck.vote_level(ev.hits, parents, [4] * 5, True, f32=True, slack=SLACK)
    assert np.array_equal(got1, ref1)


@pytest.mark.parametrize("f32", [False])
def test_inclusion_proof_catches_full_vote_pairs(orc, f32):
    """On the measured workload's level 0 and first refinement level, the
    pairs left for evaluation that still vote in every box are a small
    fraction of those the inclusion proof classified (FP64 levels: FP32
    levels run no class proofs)."""
    ev = toymc.config_event(2, 0)
    root = orc.make_box(H.LO, H.HI)
    prec = orc.FP32 if f32 else orc.FP64
    v, st = hostcheck.vote_level(ev.hits, root, [16] * 5, True, f32=f32, slack=SLACK)
    assert np.array_equal(v, orc.vote_level(ev.hits, root, [16] * 5, prec=prec, slack=SLACK))
    assert st[5] > 0 and st[4] < 0.05 * st[5]
    top = np.argsort(-v.astype(np.int64), kind="stable")[:32]
    parents = np.array([orc.box_child(root, [16] * 5, int(b)) for b in top])
    v1, st1 = hostcheck.vote_level(ev.hits, parents, [4] * 5, True, f32=f32, slack=SLACK)
    assert np.array_equal(v1, orc.vote_level(ev.hits, parents, [4] * 5, prec=prec, slack=SLACK))
    assert st1[5] > 10 * st1[2] / 16


def _topk(votes, k):
    order = np.lexsort((np.arange(votes.size), -votes.astype(np.int64)))
    return order[:k], votes[order[:k]]


@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("cfg,ev_i", [(2, 0), (4, 3), (5, 4)])
def test_pruning_keeps_selection(orc, cfg, ev_i, f32):
    """With triples pruned by their vote bounds, the top-32 boxes (votes
    desc, index asc), their votes, the maximum and the max-vote set equal the
    oracle's exhaustive level; every box holds at most its exact vote; few
    triples are evaluated."""
    ev = toymc.config_event(cfg, ev_i)
    root = orc.make_box(H.LO, H.HI)
    prec = orc.FP32 if f32 else orc.FP64
    k = 32
    levels = [(np.atleast_1d(root), [10] * 5)]
    ref0 = orc.vote_level(ev.hits, root, [10] * 5, prec=prec, slack=SLACK)
    top0, _ = _topk(ref0, k)
    levels.append((np.array([orc.box_child(root, [10] * 5, int(b)) for b in top0]), [4] * 5))
    for parents, split in levels:
        ref = orc.vote_level(ev.hits, parents, split, prec=prec, slack=SLACK)
        got, st = hostcheck.vote_level(ev.hits, parents, split, True, f32=f32, slack=SLACK, prune_k=k)
        assert np.all(got <= ref)
        ti_r, tv_r = _topk(ref, k)
        ti_g, tv_g = _topk(got, k)
        assert np.array_equal(ti_r, ti_g) and np.array_equal(tv_r, tv_g)
        vmax = ref.max()
        assert got.max() == vmax
        assert np.array_equal(np.flatnonzero(got == vmax), np.flatnonzero(ref == vmax))
        n_tr = parents.size * int(np.prod(split[:3]))
        if not f32:      # FP32 levels have no class proofs, so few triples are pruned
            assert st[6] < 0.5 * n_tr, (st[6], n_tr)


@pytest.mark.parametrize("f32", [False])
@pytest.mark.parametrize("cfg,ev_i,split", [(4, 7, [4] * 5), (5, 9, [3, 4, 2, 5, 3]), (2, 0, [4] * 5)])
def test_parent_exclusion_sound(orc, cfg, ev_i, split, f32):
    """The parent-level test (the frame and pair quantities taken as
    intervals over every child triple of a refinement parent) only drops
    (parent, hit) pairs that vote in none of the parent's child boxes: the
    level's votes equal the oracle's, with and without pruning, and the test
    drops a share of the pairs on multi-helix events."""
    ev = toymc.config_event(cfg, ev_i)
    root = orc.make_box(H.LO, H.HI)
    prec = orc.FP32 if f32 else orc.FP64
    v0 = orc.vote_level(ev.hits, root, [12] * 5, prec=prec, slack=SLACK)
    top, _ = _topk(v0, 32)
    parents = np.array([orc.box_child(root, [12] * 5, int(b)) for b in top])
    ref = orc.vote_level(ev.hits, parents, split, prec=prec, slack=SLACK)
    got, st = hostcheck.vote_level(ev.hits, parents, split, True, f32=f32, slack=SLACK, parent_filter=True)
    assert np.array_equal(got, ref), np.flatnonzero(got != ref)[:10]
    if cfg != 2:
        assert st[8] > 0.1 * parents.size * ev.n_hits
    got_p, st_p = hostcheck.vote_level(ev.hits, parents, split, True, f32=f32, slack=SLACK, prune_k=32,
                                       parent_filter=True)
    assert np.all(got_p <= ref)
    ti_r, tv_r = _topk(ref, 32)
    ti_g, tv_g = _topk(got_p, 32)
    assert np.array_equal(ti_r, ti_g) and np.array_equal(tv_r, tv_g)


@pytest.mark.parametrize("cfg,ev_i", [(2, 3), (4, 2)])
def test_parent_ranges_decide_deep_levels(orc, cfg, ev_i):
    """At FP64 refinement levels the first stage also classifies stereo
    pairs from the parent's per-sign ranges of d^Ax (exclusion with the
    outer G, inclusion with the inner G).  Down a refinement chain of the
    oracle's own top-32 boxes (12^5, then 4^5 three times) the level's votes
    equal the oracle's, and the parent ranges decide pairs."""
    ev = toymc.config_event(cfg, ev_i)
    root = orc.make_box(H.LO, H.HI)
    v = orc.vote_level(ev.hits, root, [12] * 5)
    parents, split = np.atleast_1d(root), [12] * 5
    n_decided = 0
    for lev in range(1, 4):
        top, _ = _topk(v, 32)
        parents = np.array([orc.box_child(parents[int(b) // int(np.prod(split))], split, int(b) % int(np.prod(split)))
                            for b in top])
        split = [4] * 5
        v = orc.vote_level(ev.hits, parents, split)
        got, st = hostcheck.vote_level(ev.hits, parents, split, True, parent_filter=True)
        assert np.array_equal(got, v), (lev, np.flatnonzero(got != v)[:10])
        n_decided += int(st[9])
    assert n_decided > 0


@pytest.mark.parametrize("cfg,ev_i", [(2, 1), (4, 7), (5, 4)])
def test_magnitude_bound_contains_point_drift(orc, cfg, ev_i):
    """The magnitude bound M of d^Ax over a triple (the classification's
    cheap exclusion) holds the oracle's own point evaluation: |e| <= M at the
    box centres of sampled triples (corners of the (z0, tanl) grid and random
    boxes), both drift signs, at level 0 and on refinement parents; the bound
    exists for almost every pair."""
    ev = toymc.config_event(cfg, ev_i)
    prep = orc.prep_hits(ev.hits)
    stereo = np.flatnonzero((prep["valid"] == 1) & (prep["axial"] == 0))
    root = orc.make_box(H.LO, H.HI)
    rng = np.random.default_rng(cfg * 100 + ev_i)
    v0 = orc.vote_level(ev.hits, root, [12] * 5)
    top, _ = _topk(v0, 8)
    cases = [(root, [12] * 5)] + [(orc.box_child(root, [12] * 5, int(b)), [4, 3, 5, 4, 4]) for b in top[:3]]
    n_pairs = n_bound = n_checked = 0
    for parent, split in cases:
        m012, m34 = int(np.prod(split[:3])), split[3] * split[4]
        corners = [0, split[4] - 1, m34 - split[4], m34 - 1]
        for tc in rng.choice(m012, size=min(m012, 12), replace=False):
            for hi in stereo:
                rc, M, _, _ = hostcheck.e_magnitude(ev.hits[hi], parent, split, tc)
                assert rc >= 0
                n_pairs += 1
                if rc == 0:
                    continue
                n_bound += 1
                for j in corners + list(rng.integers(0, m34, size=4)):
                    box = orc.box_child(parent, split, int(tc) * m34 + int(j))
                    c = 0.5 * (box["lo"] + box["hi"]).ravel()
                    for s in (1, -1):
                        ok, e = orc.stereo_e(prep[hi], c, s)
                        if ok:
                            n_checked += 1
                            assert abs(e) <= M, (tc, hi, j, s, e, M)
    assert n_bound >= 0.95 * n_pairs
    assert n_checked > 1000


@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("cfg,ev_i", [(2, 0), (2, 3), (4, 3), (5, 4)])
def test_tie_cut_keeps_selection(orc, cfg, ev_i, f32):
    """With the tie cut (triples after the one at which the lower bounds >= T
    first cover k boxes, and whose upper bound is exactly T, are pruned too):
    the top-32 boxes and their votes and the maximum equal the oracle's
    exhaustive level, every box holds at most its exact vote, and no more
    triples are evaluated than without the cut.  (The max-vote set is not
    kept; the cut is used only where the selection and the maximum are.)"""
    ev = toymc.config_event(cfg, ev_i)
    root = orc.make_box(H.LO, H.HI)
    prec = orc.FP32 if f32 else orc.FP64
    k = 32
    ref0 = orc.vote_level(ev.hits, root, [10] * 5, prec=prec, slack=SLACK)
    top0, _ = _topk(ref0, k)
    levels = [(np.atleast_1d(root), [10] * 5),
              (np.array([orc.box_child(root, [10] * 5, int(b)) for b in top0]), [4] * 5)]
    for li, (parents, split) in enumerate(levels):
        ref = ref0 if li == 0 else orc.vote_level(ev.hits, parents, split, prec=prec, slack=SLACK)
        got, st = hostcheck.vote_level(ev.hits, parents, split, True, f32=f32, slack=SLACK, prune_k=k, ties=True)
        _, st0 = hostcheck.vote_level(ev.hits, parents, split, True, f32=f32, slack=SLACK, prune_k=k)
        assert np.all(got <= ref)
        ti_r, tv_r = _topk(ref, k)
        ti_g, tv_g = _topk(got, k)
        assert np.array_equal(ti_r, ti_g) and np.array_equal(tv_r, tv_g)
        assert got.max() == ref.max()
        assert st[6] <= st0[6]


def test_outer_residual_contains_residual(orc):
    """The first stage's outer enclosure of G holds residual_G's interval for
    every pair: boxes at random places (phi0 ranges holding the extrema of
    the sine and not), widths from 1e-6 to 0.9 rad, hits of several events;
    and it is not much wider."""
    rng = np.random.default_rng(21)
    n_checked, worst = 0, 0.0
    events = [toymc.config_event(4, i) for i in (3, 7)] + [toymc.config_event(2, 1)]
    for trial in range(40):
        lo, hi = H.LO.copy(), H.HI.copy()
        w = 10 ** rng.uniform(-6, np.log10(0.9))
        lo[1] = rng.uniform(0, 2 * np.pi)
        hi[1] = lo[1] + w
        k = rng.uniform(-0.6, 0.5)
        lo[2], hi[2] = k, k + 10 ** rng.uniform(-4, -1)
        box = orc.make_box(lo, hi)
        ev = events[trial % len(events)]
        g = hostcheck.g_pairs(ev.hits, box, [2, 3, 2, 1, 1])
        used = np.any(g != 0, axis=2)
        assert np.all(g[..., 2][used] <= g[..., 0][used]) and np.all(g[..., 3][used] >= g[..., 1][used])
        n_checked += int(used.sum())
        worst = max(worst, float(np.max((g[..., 3] - g[..., 2]) - (g[..., 1] - g[..., 0]))))
    assert n_checked > 5000
    assert worst < 1e-12


def test_fp32_enclosure_holds_centre_values(orc):
    """The second stage's FP32 enclosure of d^Ax (outward FP32 rounding of
    the FP64 pair quantities) holds d^Ax at every box centre of the triple,
    for both drift signs, on boxes from 1e-4 of the search domain to half of
    it around a true helix of several configurations; it exists wherever the
    FP64 enclosure does and is wider by at most 1e-6 m."""
    rng = np.random.default_rng(5)
    n_pairs, worst = 0, 0.0
    for trial in range(24):
        cfg = (1, 2, 4, 5)[trial % 4]
        ev = toymc.config_event(cfg, trial // 4)
        t = ev.truth[0]
        w = (H.HI - H.LO) * 10 ** rng.uniform(-4, -0.3)
        lo = np.maximum(t - w * rng.uniform(0.1, 1, 5), H.LO)
        hi = np.minimum(t + w * rng.uniform(0.1, 1, 5), H.HI)
        o = hostcheck.encl_pairs(ev.hits, orc.make_box(lo, hi), [3, 3, 3, 8, 8]).reshape(-1, 10)
        o = o[o[:, 9] == 1]
        ok64, ok32, pts = o[:, 0] == 1, o[:, 3] == 1, o[:, 6] > 0
        assert np.all(ok32[ok64])
        m = ok32 & pts
        assert np.all(o[m, 7] >= o[m, 4]) and np.all(o[m, 8] <= o[m, 5])
        b = ok64 & ok32
        worst = max(worst, float(np.max((o[b, 5] - o[b, 4]) - (o[b, 2] - o[b, 1]), initial=0.0)))
        n_pairs += int(m.sum())
    assert n_pairs > 10000
    assert worst < 1e-6
