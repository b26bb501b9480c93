"""Pins of the oracle's window schedule pieces against geometry, brute force
and the generator's truth: the forward-hit test, the change of reference
point, the hit point about a reference point, the mirror twin, and the
recovery of noiseless helices by the whole window search.

The references here are written independently of the oracle (numpy long
double, sampling), never with its routines.
"""
import math

import numpy as np
import pytest

from paper_2401_04576_amd import toymc
from tests import _helpers as H

TWO_PI = 2.0 * math.pi


def _wrap(x):
    return (x + math.pi) % TWO_PI - math.pi


def test_forward_test_brute_force(orc):
    """Sound: if any phi0 of the box puts the hit ahead, the test says so.
    Tight: boxes entirely behind the hit (by a margin) are rejected."""
    rng = np.random.default_rng(11)
    ev = toymc.config_event(4, 1)
    pr = orc.prep_hits(ev.hits)
    n_ahead = n_behind = 0
    for _ in range(3000):
        i = int(rng.integers(len(pr)))
        w = float(10.0 ** rng.uniform(-6, math.log10(3.0)))
        a = float(rng.uniform(-2.0, 8.0))
        box = orc.make_box([-1e-3, a, 0.1, 0.0, 0.0], [1e-3, a + w, 0.2, 0.01, 0.1])
        phis = np.concatenate([[a, a + w], rng.uniform(a, a + w, 400)])
        c = np.cos(phis.astype(np.longdouble) - np.longdouble(pr[i]["phip"]))
        f = orc.forward(pr[i:i + 1], box)
        if c.max() > 0:
            assert f == 1, (i, a, w)
            n_ahead += 1
        if c.max() < -1e-9:
            assert f == 0, (i, a, w)
            n_behind += 1
    assert n_ahead > 500 and n_behind > 500


def test_forward_test_removes_the_mirror_twin(orc):
    """(d0, phi0, kappa, z0, tanl) and (-d0, phi0 + pi, -kappa, z0, -tanl) trace
    the same points: without the test a small box around each gets every
    hit; with it, only the box travelling away from the origin does."""
    for e in range(3):
        ev = toymc.config_event(3, e)
        t = np.array(ev.truth[0], dtype=float)
        twin = np.array([-t[0], (t[1] + math.pi) % TWO_PI, -t[2], t[3], -t[4]])
        h = np.array([2e-4, 2e-3, 2e-3, 2e-3, 2e-3])
        for p, fwd_votes in ((t, ev.n_hits), (twin, 0)):
            box = orc.make_box(p - h, p + h)
            assert orc.vote_level(ev.hits, box, [1] * 5)[0] == ev.n_hits
            assert orc.vote_level(ev.hits, box, [1] * 5, forward=True)[0] == fwd_votes


def _shift_ld(p, dx, dy):
    """perigee parameters about a point moved by (dx, dy), from the circle's
    centre and the arc between the two points of closest approach (long
    double; kappa != 0)"""
    d0, f0, k, z0, l = (np.longdouble(v) for v in p)
    R = 1 / k
    cx, cy = -(R + d0) * np.sin(f0), (R + d0) * np.cos(f0)
    vx, vy = cx - np.longdouble(dx), cy - np.longdouble(dy)
    rho = np.sqrt(vx * vx + vy * vy)
    sg = np.sign(k)
    f1 = np.arctan2(-sg * vx, sg * vy) % np.longdouble(TWO_PI)
    d1 = sg * rho - R
    df = (f1 - f0 + np.longdouble(math.pi)) % np.longdouble(TWO_PI) - np.longdouble(math.pi)
    return np.array([d1, f1, k, z0 + l * R * df, l], dtype=np.float64)


def test_frame_shift_matches_direct_geometry(orc):
    rng = np.random.default_rng(5)
    for _ in range(2000):
        p = np.array([rng.normal(0, 3e-3), rng.uniform(0, TWO_PI), rng.choice([-1, 1]) * rng.uniform(0.05, 0.6),
                      rng.normal(0, 0.02), rng.uniform(-0.8, 0.8)])
        r, a = rng.uniform(0.1, 0.8), rng.uniform(0, TWO_PI)
        dx, dy = r * math.cos(a), r * math.sin(a)
        q = orc.frame_shift(p, dx, dy)
        want = _shift_ld(p, dx, dy)
        assert abs(q[0] - want[0]) < 1e-12 + 1e-12 * abs(want[0])
        assert abs(_wrap(q[1] - want[1])) < 1e-12
        assert q[2] == p[2] and q[4] == p[4]
        assert abs(q[3] - want[3]) < 1e-10
        # and back
        b = orc.frame_shift(q, -dx, -dy)
        assert abs(b[0] - p[0]) < 1e-12 and abs(_wrap(b[1] - p[1])) < 1e-12 and abs(b[3] - p[3]) < 1e-10


def test_frame_shift_straight_line(orc):
    """kappa = 0: the line's distance and direction about the new point."""
    rng = np.random.default_rng(6)
    for _ in range(200):
        p = np.array([rng.normal(0, 3e-3), rng.uniform(0, TWO_PI), 0.0, rng.normal(0, 0.02), rng.uniform(-1, 1)])
        dx, dy = rng.uniform(-0.5, 0.5, 2)
        q = orc.frame_shift(p, dx, dy)
        n = np.array([-math.sin(p[1]), math.cos(p[1])])
        u = np.array([math.cos(p[1]), math.sin(p[1])])
        assert abs(q[0] - (p[0] - n @ [dx, dy])) < 1e-15
        assert abs(_wrap(q[1] - p[1])) < 1e-15
        assert abs(q[3] - (p[3] + p[4] * (u @ [dx, dy]))) < 1e-15


def test_point_G_is_the_distance_to_the_circle(orc):
    """|G| at a parameter point is, to first order, the hit point's distance
    from the circle: the closest measurement point rule ranks by it."""
    ev = toymc.config_event(3, 2)
    t = ev.truth[0]
    pr = orc.prep_hits(ev.hits)
    xc, yc, R = H.helix_circle(t)
    for i in range(len(pr)):
        dist = abs(math.hypot(pr[i]["px"] - xc, pr[i]["py"] - yc) - abs(R))
        g = abs(orc.point_G(pr[i:i + 1], t))
        assert abs(g - dist) < 0.05 * dist + 1e-9


def test_prep_about_a_reference_point(orc):
    ev = toymc.config_event(2, 1)
    p0 = orc.prep_hits(ev.hits)
    p1 = orc.prep_hits(ev.hits, ref=(0.3, -0.2))
    assert np.array_equal(p1["px"], p0["px"] - 0.3) and np.array_equal(p1["py"], p0["py"] + 0.2)
    assert np.allclose(p1["r"], np.hypot(p1["px"], p1["py"]), rtol=1e-15, atol=0)
    assert np.array_equal(p1["tant"], p0["tant"]) and np.array_equal(p1["d"], p0["d"])
    p2 = orc.prep_hits(ev.hits, ref=(0.0, 0.0))
    assert p2.tobytes() == p0.tobytes()


def _truth_in(grid, t):
    for j in range(5):
        lo, hi = grid["lo"][j], grid["hi"][j]
        x = t[j]
        if j == 1:
            c = 0.5 * (lo + hi)
            x = c + _wrap(x - c)
        if not lo <= x <= hi:
            return False
    return True


def test_window_search_recovers_noiseless_helices(orc):
    """The window schedule on noiseless single-helix events: the truth lies in
    every level's grid (in that level's frame), the level-0 maximum is every
    hit, every hit is assigned, and the helix is recovered within the
    tolerances (1 mm, 5 mrad, 0.01 /m, 10 mm, 0.02)."""
    sc = orc.make_sched(H.LO, H.HI, **toymc.WINDOW_KW)
    for e in range(2):
        ev = toymc.config_event(3, e)
        hx, ass, tr = orc.find_helices(ev.hits, sc, max_out=1, want_trace=True)
        t0 = np.array(ev.truth[0], dtype=float)
        assert len(hx) == 1
        assert tr["vmax"][0][0] == ev.n_hits
        for lev in range(sc["n_refine"] + 1):
            ref = tr["ref"][0][lev]
            t = orc.frame_shift(t0, ref[0], ref[1]) if ref.any() else t0
            assert _truth_in(tr["grid"][0][lev], t), (e, lev)
        assert hx[0]["n_assigned"] == ev.n_hits
        assert toymc.recovered(hx[0]["p"], t0), (e, hx[0]["p"], t0)
