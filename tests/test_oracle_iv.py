"""Pins of the oracle's sound whole-box arithmetic (IV levels): d^Ax
enclosed over every point of a box, with Phi enclosed through Eq.
CSAXtoPHI_a, instead of the point value at the middle of the voxel.

References: the exact-Phi point value of d^Ax (pinned against the
generator's 3-D closest approach in test_oracle_exact_phi.py) at points
sampled inside each box, and the true residual of Eq. ApoVote at such
points (G in long double from the perigee geometry).
"""
import numpy as np
import pytest

from paper_2401_04576_amd import toymc
from tests import _helpers as H


def _random_box(orc, rng, centre=None):
    w = (H.HI - H.LO) * 10.0 ** rng.uniform(-6, -1, 5)
    if centre is None:
        lo = H.LO + (H.HI - H.LO - w) * rng.random(5)
    else:
        lo = np.asarray(centre, dtype=float) - w * rng.random(5)
    return orc.make_box(lo, lo + w), lo, w


def test_iv_enclosure_holds_exact_points(orc):
    """Over boxes from 1e-6 to 1e-1 of the range, at random places and
    around generated helices, every sampled point's exact d^Ax lies in the
    box enclosure (to 1e-9 m, the point value's own rounding and its
    three-step Phi)."""
    rng = np.random.default_rng(61)
    n_in, n_ok = 0, 0
    for cfg, ev_i in ((1, 0), (2, 1), (4, 2), (5, 3)):
        ev = toymc.config_event(cfg, ev_i)
        pr = orc.prep_hits(ev.hits)
        stereo = np.flatnonzero((pr["axial"] == 0) & (pr["valid"] == 1))
        for k in range(40):
            box, lo, w = _random_box(orc, rng, ev.truth[k % len(ev.truth)] if k % 2 else None)
            for i in rng.choice(stereo, size=min(6, stereo.size), replace=False):
                for s in (1, -1):
                    ok, elo, ehi = orc.stereo_encl(pr[i], box, s)
                    if not ok:
                        continue
                    n_ok += 1
                    for _ in range(12):
                        p = lo + w * rng.random(5)
                        okp, e = orc.stereo_e(pr[i], p, s, exact=True)
                        if okp:
                            assert elo - 1e-9 <= e <= ehi + 1e-9, (cfg, k, i, s, elo, e, ehi)
                            n_in += 1
    assert n_ok > 1000 and n_in > 10000


def test_iv_vote_is_sound_against_the_true_residual(orc):
    """P4 on the true residual: where 2G - 2e - kappa e^2, with the exact d^Ax
    and G in long double, changes sign among points sampled in a box (for a
    drift sign), the IV vote of that box is cast."""
    rng = np.random.default_rng(62)
    n_change = 0
    for cfg, ev_i in ((1, 1), (2, 2), (4, 3)):
        ev = toymc.config_event(cfg, ev_i)
        pr = orc.prep_hits(ev.hits)
        stereo = np.flatnonzero((pr["axial"] == 0) & (pr["valid"] == 1))
        for k in range(60):
            t = np.asarray(ev.truth[k % len(ev.truth)], dtype=float)
            box, lo, w = _random_box(orc, rng, t)
            for i in rng.choice(stereo, size=min(8, stereo.size), replace=False):
                for s in (1, -1):
                    vals = []
                    for _ in range(16):
                        p = lo + w * rng.random(5)
                        okp, e = orc.stereo_e(pr[i], p, s, exact=True)
                        if not okp:
                            continue
                        G = H.G_ld(p, pr[i]["r"], pr[i]["phip"])
                        e = np.longdouble(e)
                        vals.append(2 * G - 2 * e - np.longdouble(p[2]) * e * e)
                    if vals and min(vals) < 0 < max(vals):
                        n_change += 1
                        assert orc.pair_vote_iv(pr[i], box) == 1, (cfg, k, i, s)
    assert n_change > 50


def test_iv_truth_box_collects_all_hits(orc):
    """A box around the truth of a noiseless event gets every hit at every
    width, and its d^Ax enclosures shrink with the box."""
    for ev_i in range(3):
        ev = toymc.config_event(1, ev_i)
        t = np.array(ev.truth[0], dtype=float)
        pr = orc.prep_hits(ev.hits)
        i = int(np.flatnonzero(pr["axial"] == 0)[0])
        widths = []
        for w in (1e-2, 1e-4, 1e-6):
            h = w * np.array([5e-3, 1.0, 0.5, 5e-2, 0.5])
            box = orc.make_box(t - h, t + h)
            assert orc.vote_level(ev.hits, box, [1] * 5, prec=orc.IV)[0] == ev.n_hits, (ev_i, w)
            ok, lo, hi = orc.stereo_encl(pr[i], box, 1)
            assert ok
            widths.append(hi - lo)
        assert widths[0] > 50 * widths[1] > 2500 * widths[2]


def test_iv_level_contains_most_midvoxel_votes(orc):
    """On a level-0 grid the IV votes hold the mid-voxel votes except where
    the mid-voxel value itself lies off the exact d^Ax (the ApproxPhi error,
    ~1e-7 m): at most a few boxes in 10^4 lose a vote, and the IV level
    casts more votes overall (it is the sound, wider test)."""
    ev = toymc.config_event(2, 5)
    root = orc.make_box(H.LO, H.HI)
    v64 = orc.vote_level(ev.hits, root, [8] * 5)
    viv = orc.vote_level(ev.hits, root, [8] * 5, prec=orc.IV)
    d = viv.astype(np.int64) - v64
    assert (d < 0).mean() < 1e-3
    assert viv.sum() > v64.sum()
    assert viv.max() >= v64.max()


@pytest.mark.slow
def test_window_search_with_iv_levels_recovers(orc):
    """The default window schedule with its last level sound (IV)
    recovers a noiseless single-helix event."""
    kw = dict(toymc.WINDOW_KW)
    kw["prec"] = [orc.FP64] * 7 + [orc.IV]
    sc = orc.make_sched(H.LO, H.HI, **kw)
    ev = toymc.config_event(3, 0)
    hx, _ = orc.find_helices(ev.hits, sc, max_out=1)
    assert len(hx) == 1 and hx[0]["n_assigned"] == ev.n_hits
    assert toymc.recovered(hx[0]["p"], ev.truth[0]), (hx[0]["p"], ev.truth[0])
