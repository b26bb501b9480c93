"""Enclosure pins of the oracle's vote predicate (Eq. ApoVote, kappa-scaled).

P4: for random boxes (widths 1e-6 .. 1e-1 of the search range) and hits of
generated events, the residual 2G(p) - 2e - kappa e^2, evaluated in long
double at random points p of the box and drift values e in the tolerance
band around the point-evaluated d^Ax, lies inside the oracle's interval, and
G(p) inside the G interval.
P7: on tiny grids around the truth, a sampled sign change of the residual
inside a box implies a vote (the level loop, the index order and the
predicate agree), and the over-vote rate is reported.
"""
import numpy as np

from paper_2401_04576_amd import toymc
from tests import _helpers as H


def _residual(p, e, r, phip):
    G = H.G_ld(p, r, phip)
    e = np.longdouble(e)
    return G, 2 * G - 2 * e - np.longdouble(p[2]) * e * e


def test_enclosure_contains_sampled_residuals(orc):
    rng = np.random.default_rng(21)
    span = H.HI - H.LO
    n_checked = 0
    for ev_i in range(6):
        ev = toymc.config_event(2 if ev_i % 2 else 1, ev_i)
        pr = orc.prep_hits(ev.hits)
        t = ev.truth[0]
        for _ in range(12):
            frac = np.exp(rng.uniform(np.log(1e-6), np.log(1e-1), 5))
            w = frac * span
            centre = t + rng.uniform(-0.5, 0.5, 5) * w * 3
            box = orc.make_box(centre - w / 2, centre + w / 2)
            P = rng.uniform(box["lo"], box["hi"], size=(400, 5))
            for i in rng.choice(len(pr), size=6, replace=False):
                v, dbg = orc.pair_vote(pr[i], box, debug=True)
                Glo, Ghi = dbg[0], dbg[1]
                for si in range(2):
                    e = dbg[6 + si]
                    if not np.isfinite(e):
                        continue
                    Hlo, Hhi = dbg[2 + 2 * si], dbg[3 + 2 * si]
                    band = pr[i]["band"]
                    es = rng.uniform(e - band, e + band, P.shape[0]) if band > 0 else np.full(P.shape[0], e)
                    for p, ee in zip(P, es):
                        G, Hm = _residual(p, ee, pr[i]["r"], pr[i]["phip"])
                        assert Glo <= G <= Ghi
                        assert Hlo <= Hm <= Hhi
                    n_checked += P.shape[0]
                    if Hlo <= 0 <= Hhi:
                        assert v == 1
    assert n_checked > 50000


def test_tiny_grid_sign_change_implies_vote(orc):
    """Brute force on 4^5 tiny boxes around the truth (noiseless events)."""
    rng = np.random.default_rng(22)
    over = []
    for ev_i in range(2):
        ev = toymc.config_event(1, ev_i)
        pr = orc.prep_hits(ev.hits)
        t = ev.truth[0]
        w = (H.HI - H.LO) * 2e-4
        parent = orc.make_box(t - 2 * w + rng.uniform(-0.5, 0.5, 5) * w, t + 2 * w)
        split = [4] * 5
        votes = orc.vote_level(ev.hits, parent, split)
        for b in rng.choice(4 ** 5, size=64, replace=False):
            box = orc.box_child(parent, split, b)
            c = 0.5 * (box["lo"] + box["hi"])
            P = rng.uniform(box["lo"], box["hi"], size=(300, 5))
            brute = 0
            for i in range(len(pr)):
                hit_votes = False
                for s in (1, -1):
                    ok, e = orc.stereo_e(pr[i], c, s)
                    if not ok:
                        continue
                    vals = np.array([_residual(p, e, pr[i]["r"], pr[i]["phip"])[1] for p in P])
                    if vals.min() <= 0 <= vals.max():
                        hit_votes = True
                brute += hit_votes
            assert votes[b] >= brute
            over.append(int(votes[b]) - brute)
    # the pessimism of the enclosure is reported, not bounded
    print("mean over-votes per box", float(np.mean(over)))
