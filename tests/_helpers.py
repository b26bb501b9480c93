"""Shared test helpers: grid ranges, schedules and independent reference maths.

Nothing here calls the HIP library; the independent references use numpy
long double (64-bit mantissa) or mpmath, never the oracle's routines.
"""
import math

import numpy as np

from paper_2401_04576_amd import toymc

LO = np.array(toymc.GRID_RANGE_LO)
HI = np.array(toymc.GRID_RANGE_HI)


def make_hits(rows):
    h = np.zeros(len(rows), dtype=toymc.HIT_DTYPE)
    for i, r in enumerate(rows):
        h[i] = tuple(float(v) for v in r)
    return h


def axial_hit(px, py, drift, band=0.0):
    return (px, py, -1.0, px, py, 1.0, drift, band)


def stereo_wire_through(helix, s, d, tan_tau, side=1.0):
    """A wire at distance d from helix point s, perpendicular to the helix
    tangent there, stereo slope tan_tau in the tangential direction.
    Returns the hit row (end points at z = +-1) and the signed drift sign."""
    x, y, z = toymc.helix_point(helix, s)
    T = np.array(toymc.helix_tangent(helix, s), dtype=float)
    ph = math.atan2(y, x)
    W = np.array([-math.sin(ph) * tan_tau, math.cos(ph) * tan_tau, 1.0])
    n = np.cross(T, W)
    n /= np.linalg.norm(n)
    M = np.array([x, y, z]) + side * d * n
    # line point at height zz: M + (zz - M_z) W  (W has unit z component)
    a = M + (-1.0 - M[2]) * W
    b = M + (1.0 - M[2]) * W
    return (a[0], a[1], -1.0, b[0], b[1], 1.0, d, 0.0)


def G_ld(p, r, phip):
    """kappa (|P - C|^2 - R^2) / 2 in perigee variables, long double."""
    d0, phi0, kap = (np.longdouble(v) for v in p[:3])
    r = np.longdouble(r)
    return (kap / 2) * (r * r + d0 * d0) + (1 + kap * d0) * r * np.sin(phi0 - np.longdouble(phip)) + d0


def helix_circle(p):
    d0, phi0, kap = p[:3]
    R = 1.0 / kap
    return -(R + d0) * math.sin(phi0), (R + d0) * math.cos(phi0), R


def full_sched(orc, bins=(16,) * 5, n_refine=4, top_k=32, split=(4,) * 5, v_min=10, n_helix_max=1):
    return orc.make_sched(LO, HI, bins, n_refine=n_refine, top_k=top_k, split=split, v_min=v_min,
                          n_helix_max=n_helix_max)
