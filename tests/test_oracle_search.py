"""Pins of the oracle's level loop, selection, split and estimate.

P11: top-k against numpy's lexsort; the child-box tiling against its
definition; the estimate against an independent numpy implementation.
P5/P6: on noiseless tracks the cell containing the truth collects every hit
at every refinement width, and it is among the max-vote cells at level 0.
P8: hit order does not change votes.
"""
import math

import numpy as np
import pytest

from paper_2401_04576_amd import toymc
from tests import _helpers as H


def test_topk_matches_lexsort(orc):
    rng = np.random.default_rng(31)
    for n, vmax in [(1, 3), (7, 2), (1000, 3), (50000, 20), (4096, 1)]:
        v = rng.integers(0, vmax + 1, n).astype(np.uint16)
        for k in (1, 5, 32, 64):
            idx, vv = orc.topk(v, k)
            ref = np.lexsort((np.arange(n), -v.astype(np.int64)))[:k]
            assert np.array_equal(idx, ref) and np.array_equal(vv, v[ref])


def test_children_tile_parent(orc):
    rng = np.random.default_rng(32)
    for _ in range(20):
        lo = rng.uniform(-1, 1, 5)
        hi = lo + np.exp(rng.uniform(-20, 1, 5))
        parent = orc.make_box(lo, hi)
        split = rng.integers(1, 6, 5)
        n = int(np.prod(split))
        kids = [orc.box_child(parent, split, c) for c in range(n)]
        for c, kid in enumerate(kids):
            k = np.unravel_index(c, split)          # d0 slowest, tanl fastest
            for j in range(5):
                w = (hi[j] - lo[j]) / split[j]
                assert kid["lo"][j] == lo[j] + k[j] * w
                assert kid["hi"][j] == (hi[j] if k[j] + 1 == split[j] else lo[j] + (k[j] + 1) * w)
                if k[j] + 1 < split[j]:             # neighbours share the edge bit for bit
                    k2 = list(k)
                    k2[j] += 1
                    assert kids[int(np.ravel_multi_index(k2, split))]["lo"][j] == kid["hi"][j]


def _estimate_ref(orc, parents, split, votes, vmax):
    nc = int(np.prod(split))
    boxes = [orc.box_child(parents[b // nc], split, b % nc) for b in np.flatnonzero(votes == vmax)]
    lo = np.array([b["lo"] for b in boxes])
    hi = np.array([b["hi"] for b in boxes])
    c = 0.5 * (lo + hi)
    dv = c[:, 1] - c[0, 1]
    shift = np.where(dv > math.pi, -2 * math.pi, np.where(dv <= -math.pi, 2 * math.pi, 0.0))
    p = c.mean(axis=0)
    p[1] = (c[0, 1] + np.mean(dv + shift)) % (2 * math.pi)
    lo[:, 1] += shift
    hi[:, 1] += shift
    return p, 0.5 * (hi.max(axis=0) - lo.min(axis=0)), len(boxes)


def test_estimate_matches_independent_mean(orc):
    rng = np.random.default_rng(33)
    for trial in range(12):
        if trial % 3 == 0:       # a max-vote set straddling phi0 = 0 = 2 pi
            parents = np.array([orc.make_box([0, 2 * math.pi - 0.3, 0, 0, 0], [1, 2 * math.pi, 1, 1, 1]),
                                orc.make_box([0, 0.0, 0, 0, 0], [1, 0.3, 1, 1, 1])])
        else:
            lo = rng.uniform(-1, 1, (3, 5))
            lo[:, 1] = rng.uniform(0, 6, 3)
            parents = np.array([orc.make_box(l, l + rng.uniform(0.01, 0.2, 5)) for l in lo])
        split = [2, 3, 2, 2, 1]
        votes = rng.integers(0, 4, len(parents) * 24).astype(np.uint16)
        vmax = votes.max()
        p, err, n = orc.estimate(parents, split, votes, vmax)
        pr, er, nr = _estimate_ref(orc, parents, split, votes, vmax)
        assert n == nr
        assert np.allclose(p, pr, rtol=1e-13, atol=1e-14), (p, pr)
        assert np.array_equal(err, er) or np.allclose(err, er, rtol=0, atol=1e-15)


def _truth_cell(t, level):
    """The cell of the uniform grid (16 * 4^level per dimension) holding t."""
    n = 16 * 4 ** level
    w = (H.HI - H.LO) / n
    k = np.floor((t - H.LO) / w)
    lo = H.LO + k * w
    return lo, lo + w


@pytest.mark.parametrize("ev_i", range(4))
def test_truth_cell_collects_all_hits(orc, ev_i):
    """P5: noiseless tracks vote for the cell holding the truth at every level width."""
    ev = toymc.config_event(1, ev_i)
    t = ev.truth[0]
    for level in range(5):
        lo, hi = _truth_cell(t, level)
        votes = orc.vote_level(ev.hits, orc.make_box(lo, hi), [1] * 5)
        assert votes[0] == ev.n_hits, (level, votes[0], ev.n_hits)


def test_truth_in_level0_argmax(orc):
    """P6 at level 0 (8^5 grid for speed): the truth's cell has the max votes."""
    for ev_i in range(3):
        ev = toymc.config_event(1, ev_i)
        t = ev.truth[0]
        votes = orc.vote_level(ev.hits, orc.make_box(H.LO, H.HI), [8] * 5)
        k = np.floor((t - H.LO) / ((H.HI - H.LO) / 8)).astype(int)
        b = int(np.ravel_multi_index(k, [8] * 5))
        assert votes[b] == votes.max() == ev.n_hits


def test_hit_permutation_invariance(orc):
    ev = toymc.config_event(2, 7)
    rng = np.random.default_rng(34)
    v1 = orc.vote_level(ev.hits, orc.make_box(H.LO, H.HI), [6] * 5)
    v2 = orc.vote_level(ev.hits[rng.permutation(ev.n_hits)], orc.make_box(H.LO, H.HI), [6] * 5)
    assert np.array_equal(v1, v2)


def test_invalid_hits_never_vote(orc):
    ev = toymc.config_event(1, 3)
    hits = ev.hits.copy()
    bad = np.concatenate([hits[:4]])
    bad[0]["drift"] = -1.0                 # negative drift
    bad[1]["z1"] = bad[1]["z0"]            # zero-length wire
    bad[2]["x0"] = np.nan                  # NaN
    bad[3]["y1"] = np.inf                  # inf
    both = np.concatenate([hits, bad])
    v1 = orc.vote_level(hits, orc.make_box(H.LO, H.HI), [5] * 5)
    v2 = orc.vote_level(both, orc.make_box(H.LO, H.HI), [5] * 5)
    assert np.array_equal(v1, v2)
    assert orc.prep_hits(bad)["valid"].sum() == 0


def test_driver_stop_rule_applies_to_level0(orc):
    """The greedy loop stops only when the level-0 maximum is below v_min; a
    lower maximum at a refinement level still records the helix."""
    ev = toymc.config_event(1, 2)
    kw = dict(bins=[6] * 5, n_refine=2, top_k=4, split=[2] * 5, n_helix_max=3)
    hel, ass, tr = orc.find_helices(ev.hits, orc.make_sched(H.LO, H.HI, v_min=10, **kw), want_trace=True)
    assert tr["vmax"][0][0] >= 10 and len(hel) >= 1
    assert hel[0]["votes"] == tr["vmax"][0][2]
    assert (ass >= 0).sum() == sum(h["n_assigned"] for h in hel)
    # a level-0 maximum below v_min records nothing
    hel2, ass2 = orc.find_helices(ev.hits, orc.make_sched(H.LO, H.HI, v_min=ev.n_hits + 1, **kw))
    assert len(hel2) == 0 and (ass2 == -1).all()
