"""Pins of the oracle's exact-Phi arithmetic (IA_FP64X): Phi from Eq.
CSAXtoPHI_a by fixed-point steps instead of the second-order Eq. ApproxPhi.

The references are the generator's independent 3-D closest approach (golden
section plus Newton on the wire and the helix) and long-double evaluations
of the equation from the oracle's own intermediates, never the oracle's
routines themselves.
"""
import math

import numpy as np
import pytest

from paper_2401_04576_amd import toymc
from tests import _helpers as H


def _tangency_residuals(orc, exact, n_events=6):
    worst = 0.0
    for ev_i in range(n_events):
        ev = toymc.config_event(1, ev_i)
        pr = orc.prep_hits(ev.hits)
        t = ev.truth[0]
        xc, yc, R = H.helix_circle(t)
        for i in np.flatnonzero(pr["axial"] == 0):
            dist = math.hypot(pr[i]["px"] - xc, pr[i]["py"] - yc)
            res = min(abs(abs(R + orc.stereo_e(pr[i], t, s, exact=exact)[1]) - dist) for s in (1, -1))
            worst = max(worst, res)
    return worst


def test_exact_phi_tangency_at_truth(orc):
    """At the true helix the virtual drift circle of every stereo hit is
    tangent to the base circle: with the exact Phi to 1e-12 m (the drift is
    the generator's exact 3-D closest distance), where ApproxPhi leaves its
    O(tan^3 tau) error of ~1e-7 m."""
    exact = _tangency_residuals(orc, True)
    approx = _tangency_residuals(orc, False)
    assert exact < 1e-12, exact
    assert approx > 1e-8, approx


def _controlled(orc, helix, s_arc, d, tan_tau, side):
    row = H.stereo_wire_through(helix, s_arc, d, tan_tau, side)
    pr = orc.prep_hits(H.make_hits([row]))[0]
    xc, yc, R = H.helix_circle(helix)
    best = None
    for sg in (1, -1):
        ok, e, dbg = orc.stereo_e(pr, helix, sg, debug=True, exact=True)
        D = dict(zip(orc.STEREO_DEBUG_NAMES, dbg))
        res = abs(abs(R + e) - math.hypot(pr["px"] - xc, pr["py"] - yc))
        if best is None or res < best[0]:
            best = (res, D, sg)
    return best, pr


def test_exact_phi_is_the_closest_approach():
    """Phi - Phi^Ax from the fixed point equals the generator's closest
    approach (kappa s - phi^Ax + phi0) to 1e-11 rad at every stereo angle up to
    0.1 rad, where ApproxPhi's error grows as tan^3 tau."""
    import oracle as orc
    rng = np.random.default_rng(31)
    worst = 0.0
    for trial in range(16):
        helix = toymc.draw_helix(rng)
        helix[2] = abs(helix[2])
        s_arc = toymc.crossing_arc(helix, rng.uniform(0.3, 0.8))
        d = rng.uniform(1e-3, 8e-3)
        side = 1.0 if trial % 2 else -1.0
        for tau in (0.01, 0.04, 0.1):
            (res, D, _), pr = _controlled(orc, helix, s_arc, d, math.tan(tau), side)
            eps_exact = helix[2] * s_arc - D["dphi"]
            worst = max(worst, abs(D["eps"] - eps_exact))
            assert res < 1e-12, (trial, tau, res)
    assert worst < 1e-11, worst


def test_exact_phi_is_a_fixed_point():
    """The returned Phi satisfies Eq. CSAXtoPHI_a re-evaluated in long double
    from the oracle's intermediates (c^tau, z^St, delta, c^Ax, s^Ax, R^Ax) on
    random points near generated helices, to 1e-9 rad: the map contracts by
    about |tan(tau) tanl| R / R^Ax (~0.03 here) per step and ApproxPhi starts
    within ~5e-6 rad, so three steps leave ~1e-10 rad (d^Ax, stationary in
    Phi, moves by its square), while a wrong term in the equation moves Phi by
    ~1e-4 rad."""
    import oracle as orc
    rng = np.random.default_rng(32)
    n = 0
    for ev_i in range(4):
        ev = toymc.config_event(2, ev_i)
        pr = orc.prep_hits(ev.hits)
        t = np.array(ev.truth[0], dtype=float)
        for i in np.flatnonzero(pr["axial"] == 0):
            c = t + rng.normal(0, 1, 5) * [1e-3, 3e-3, 2e-2, 1e-2, 2e-2]
            for s in (1, -1):
                ok, e, dbg = orc.stereo_e(pr[i], c, s, debug=True, exact=True)
                if not ok:
                    continue
                D = {k: np.longdouble(v) for k, v in zip(orc.STEREO_DEBUG_NAMES, dbg)}
                tt = np.longdouble(pr[i]["tant"])
                lam = np.longdouble(c[4])
                stau = -lam * D["delta"] * D["cAx"] - D["zS"] * D["sAx"]
                rhs = np.arctan2(stau * tt, D["RAx"] ** 2 + D["ctau"] * tt)
                assert abs(rhs - D["eps"]) < 1e-9, (ev_i, i, s, float(rhs - D["eps"]))
                n += 1
    assert n > 100


def test_exact_and_approx_agree_to_third_order(orc):
    """Near the truth the two forms of d^Ax differ by less than the ApproxPhi
    error bound seen at the truth (1e-6 m)."""
    for ev_i in range(3):
        ev = toymc.config_event(1, ev_i)
        pr = orc.prep_hits(ev.hits)
        t = ev.truth[0]
        for i in np.flatnonzero(pr["axial"] == 0):
            for s in (1, -1):
                a = orc.stereo_e(pr[i], t, s)[1]
                b = orc.stereo_e(pr[i], t, s, exact=True)[1]
                assert abs(a - b) < 1e-6


def test_exact_votes_truth_cell_collects_all_hits(orc):
    """IA_FP64X levels: a cell around the truth gets every hit of a noiseless
    event at every width, as with ApproxPhi."""
    for ev_i in range(3):
        ev = toymc.config_event(1, ev_i)
        t = np.array(ev.truth[0], dtype=float)
        for w in (1e-2, 1e-4, 1e-6):
            h = w * np.array([5e-3, 1.0, 0.5, 5e-2, 0.5])
            box = orc.make_box(t - h, t + h)
            assert orc.vote_level(ev.hits, box, [1] * 5, prec=orc.FP64X)[0] == ev.n_hits, (ev_i, w)


@pytest.mark.slow
def test_window_search_with_exact_phi_recovers(orc):
    """The default window schedule with the exact Phi at its last two levels
    recovers a noiseless single-helix event."""
    kw = dict(toymc.WINDOW_KW)
    kw["prec"] = [orc.FP64] * 6 + [orc.FP64X] * 2
    sc = orc.make_sched(H.LO, H.HI, **kw)
    for e in range(1):
        ev = toymc.config_event(3, e)
        hx, ass = orc.find_helices(ev.hits, sc, max_out=1)
        assert len(hx) == 1 and hx[0]["n_assigned"] == ev.n_hits
        assert toymc.recovered(hx[0]["p"], ev.truth[0]), (e, hx[0]["p"], ev.truth[0])
