"""The margin of the class proofs against the point evaluation's rounding.

The enclosures of d^Ax over a triple (and over a parent) are widened by
1e-9 |e| + 1e-12 m so that they hold the FP64 point value every box computes,
not only the exact value of the same formula.  This checks the FP64 point
evaluation (the oracle's, which the kernels reproduce bit for bit) against
the same formula in long double (64-bit significand), with the library
transcendentals replaced by long-double ones, at points across the search
range and near generated helices: wherever the discriminant of Eq.
defdiAX_b is above A^2 / 4 (the only place the kernels decide pairs from an
enclosure) the difference stays below 1 % of the margin.
"""
import numpy as np

from paper_2401_04576_amd import toymc
from tests import _helpers as H

L = np.longdouble


def _e_longdouble(p, c, s):
    """d^Ax in long double, the oracle's operation sequence (ApproxPhi)."""
    kap, sig = L(c[2]), L(1)
    if kap < 0:
        sig = L(-1)
    if kap == 0:
        kap, sig = L(2.0 ** -30), L(1)
    dS = L(s) * L(p["d"])
    if p["axial"]:
        return True, sig * dS, None, None
    kp, d0p = sig * kap, sig * L(c[0])
    sp0, cp0 = sig * np.sin(L(c[1])), np.cos(L(c[1]))
    R = 1 / kp
    Rd = R + d0p
    xc, yc = -(Rd * sp0), Rd * cp0
    py, cps, sps = sig * L(p["py"]), sig * L(p["cphis"]), L(p["sphis"])
    Dx, Dy = L(p["px"]) - xc, py - yc
    RAx = np.sqrt(Dx * Dx + Dy * Dy)
    cAx, sAx = Dx * sps - Dy * cps, Dx * cps + Dy * sps
    sinA, cosA = sAx / RAx, cAx / RAx
    dphi = np.arctan2(Dx * cp0 + Dy * sp0, Dx * sp0 - Dy * cp0)
    z0, lam, tt = L(c[3]), L(c[4]), L(p["tant"])
    sArc = R * dphi
    zA = z0 + lam * sArc
    Phi1 = -(zA * sinA + (lam * dS) * cosA) / RAx
    c2, s2 = cosA * cosA - sinA * sinA, 2 * sinA * cosA
    Phi2 = ((lam * R) * zA - ((lam * zA) * (R - 2 * dS)) * c2
            + (zA * zA + dS * (RAx + (lam * lam) * ((R + RAx) - dS))) * s2) / (2 * (RAx * RAx))
    t2 = tt * tt
    eps = Phi1 * tt + Phi2 * t2
    se, ce = np.sin(eps), np.cos(eps)
    sinP, cosP = sinA * ce + cosA * se, cosA * ce - sinA * se
    u = np.sqrt(((1 + ((2 * lam) * sinP) * tt) + (lam * lam) * t2) + (cosP * cosP) * t2)
    delta = dS / u
    sperp = R * (dphi + eps)
    zS = (z0 + lam * sperp) - (delta * cosP) * tt
    ctau = zS * cAx - (lam * delta) * sAx
    a1, a2 = zS * tt, (lam * delta) * tt
    Q = ((2 * ctau) * tt + a1 * a1) + a2 * a2
    A = R + delta
    disc = A * A - Q
    if not disc >= 0:
        return False, None, disc, A
    return True, sig * (delta - Q / (A + np.sqrt(disc))), disc, A


def _points(rng, ev, n_rand):
    lo, hi = np.asarray(H.LO, dtype=float), np.asarray(H.HI, dtype=float)
    pts = [lo + (hi - lo) * rng.random(5) for _ in range(n_rand)]
    for t in ev.truth:
        t = np.asarray(t, dtype=float)
        for scale in (1e-4, 1e-2, 1.0):
            pts.append(t + scale * rng.normal(0, 1, 5) * [1e-3, 3e-2, 5e-2, 1e-2, 5e-2])
    return pts


def test_point_rounding_far_inside_the_margin(orc):
    rng = np.random.default_rng(41)
    worst, n_checked, n_ill = 0.0, 0, 0
    for cfg, idx in ((1, range(3)), (2, range(3)), (4, range(3)), (5, range(2))):
        for i in idx:
            ev = toymc.config_event(cfg, i)
            pr = orc.prep_hits(ev.hits)
            stereo = np.flatnonzero(pr["axial"] == 0)
            for c in _points(rng, ev, 12):
                for h in rng.choice(stereo, size=min(12, stereo.size), replace=False):
                    for s in (1, -1):
                        ok64, e64 = orc.stereo_e(pr[h], c, s)
                        okl, el, disc, A = _e_longdouble(pr[h], c, s)
                        if not (okl and ok64):
                            continue
                        if not (A > 0 and disc > A * A / 4):
                            n_ill += 1
                            continue
                        margin = 1e-9 * abs(float(el)) + 1e-12
                        worst = max(worst, abs(float(L(e64) - el)) / margin)
                        n_checked += 1
    print(f"{n_checked} points, largest rounding error {worst:.2e} of the margin, {n_ill} ill-conditioned")
    assert n_checked > 3000
    assert worst < 0.01, worst
    # on this chamber every evaluated point is well conditioned
    assert n_ill <= n_checked // 100, (n_ill, n_checked)


def test_magnitude_bound_widening_covers_its_rounding():
    """The magnitude bound of d^Ax (first classification stage) is a chain of
    at most ~60 sums, products, quotients and roots of non-negative numbers,
    each rounded to nearest (relative error <= 2^-53), so its relative error
    is below 60 * 2^-53 < 2^-46, far inside its 2^-29 widening."""
    from fractions import Fraction
    growth = (1 + Fraction(1, 2 ** 53)) ** 60 - 1       # exact compounding of 60 roundings
    assert growth < Fraction(1, 2 ** 46) < Fraction(1, 2 ** 29)
