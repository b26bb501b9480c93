"""Seeded synthetic drift-chamber events (input generator only).

This module produces the inputs of the helix search: wire end points, drift
radii and tolerance bands, plus the generator truth.  It holds none of the
vote arithmetic (no Apollonius residual, no interval code, no stereo
correction): drift radii are found by direct numerical minimisation of the
3-D helix-to-wire distance, which is how the paper defines a hit (Sec. 3.2:
a hit is a drift distance, the smallest wire-helix distance, together with
the wire end points).

Geometry (a synthetic stand-in for the paper's private COMET-like toy model,
Sec. 3.2, which does not ship): a cylindrical chamber of 20 layers at radii
0.20..0.80 m, 64..256 wires per layer, wires 2 m long (z in [-1, 1]), stereo
angle alternating 0 / +60 / -60 mrad by superlayer of 4 layers, B = 1 T along z.

Helix parametrisation (perigee about the origin, the paper's first reference
point, Sec. 3.3): d0, phi0, kappa, z0, tanl.  The centre of the transverse
circle is C = (R + d0)(-sin phi0, cos phi0) with signed R = 1/kappa, the point
at transverse arc length s is C + R (sin(phi0 + kappa s), -cos(phi0 + kappa s)),
z = z0 + tanl s (Eqs. HelixEq_a-c).  kappa > 0 turns counter-clockwise seen
from +z, so a positive charge in B = +z has kappa = -0.299792458 B / pT < 0.

Every draw comes from numpy's PCG64 seeded with SeedSequence([config, event]).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

HIT_DTYPE = np.dtype([("x0", "f8"), ("y0", "f8"), ("z0", "f8"),
                      ("x1", "f8"), ("y1", "f8"), ("z1", "f8"),
                      ("drift", "f8"), ("band", "f8")])

C_LIGHT = 0.299792458  # GeV / (T m)


# --------------------------------------------------------------------------
# chamber
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Chamber:
    n_layers: int = 20
    r_min: float = 0.20
    r_max: float = 0.80
    half_length: float = 1.0
    b_field: float = 1.0
    stereo_mrad: tuple = (0.0, 60.0, -60.0, 0.0, 60.0)   # per superlayer of 4

    def radius(self, layer):
        return self.r_min + np.asarray(layer) * (self.r_max - self.r_min) / (self.n_layers - 1)

    def n_wires(self, layer):
        layer = np.asarray(layer)
        return (64 + np.floor(192.0 * layer / (self.n_layers - 1) + 0.5)).astype(np.int64)

    def tan_tau(self, layer):
        sl = np.asarray(layer) // 4
        return np.tan(np.asarray(self.stereo_mrad)[sl] * 1e-3)

    def wire_phi(self, layer, j):
        layer = np.asarray(layer)
        return 2.0 * np.pi * (np.asarray(j) + 0.5 * (layer % 2)) / self.n_wires(layer)

    def half_cell(self, layer):
        return np.pi * self.radius(layer) / self.n_wires(layer)

    def wire_geometry(self, layer, j):
        """Wire through P (at z = 0) with transverse slope t = dxy/dz."""
        r = self.radius(layer)
        phw = self.wire_phi(layer, j)
        tt = self.tan_tau(layer)
        px, py = r * np.cos(phw), r * np.sin(phw)
        tx, ty = -np.sin(phw) * tt, np.cos(phw) * tt
        return px, py, tx, ty

    def wire_endpoints(self, layer, j):
        px, py, tx, ty = self.wire_geometry(layer, j)
        L = self.half_length
        return (px - L * tx, py - L * ty, -L + 0.0 * px,
                px + L * tx, py + L * ty, L + 0.0 * px)

    @property
    def total_wires(self):
        return int(np.sum(self.n_wires(np.arange(self.n_layers))))


CHAMBER = Chamber()


# --------------------------------------------------------------------------
# helix geometry (HelixEq_a-c in perigee form)
# --------------------------------------------------------------------------
def helix_centre(d0, phi0, kappa):
    R = 1.0 / kappa
    return -(R + d0) * np.sin(phi0), (R + d0) * np.cos(phi0), R


def helix_point(p, s):
    d0, phi0, kappa, z0, tanl = p
    xc, yc, R = helix_centre(d0, phi0, kappa)
    th = phi0 + kappa * s
    return xc + R * np.sin(th), yc - R * np.cos(th), z0 + tanl * s


def helix_tangent(p, s):
    _, phi0, kappa, _, tanl = p
    th = phi0 + kappa * s
    return np.cos(th), np.sin(th), tanl + 0.0 * th


def crossing_arc(p, radius):
    """Smallest s > 0 at which the transverse helix reaches `radius` (NaN if never)."""
    d0, phi0, kappa, _, _ = p
    xc, yc, R = helix_centre(d0, phi0, kappa)
    s_hi = np.pi * abs(R)

    def rho(s):
        x, y, _ = helix_point(p, s)
        return math.hypot(x, y)

    if rho(s_hi) < radius or abs(d0) > radius:
        return float("nan")
    lo, hi = 0.0, s_hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if rho(mid) < radius:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15:
            break
    return 0.5 * (lo + hi)


def _line_terms(p, s, px, py, tx, ty):
    x, y, z = helix_point(p, s)
    n = math.sqrt(tx * tx + ty * ty + 1.0)
    wx, wy, wz = tx / n, ty / n, 1.0 / n
    gx, gy, gz = x - px, y - py, z
    gw = gx * wx + gy * wy + gz * wz
    return (gx, gy, gz), (wx, wy, wz), gw


def helix_line_distance(p, s, px, py, tx, ty):
    """Distance from helix point s to the line {(px + z tx, py + z ty, z)}; also the wire z."""
    (gx, gy, gz), (wx, wy, wz), gw = _line_terms(p, s, px, py, tx, ty)
    qx, qy, qz = gx - gw * wx, gy - gw * wy, gz - gw * wz
    return math.sqrt(qx * qx + qy * qy + qz * qz), gw * wz


def closest_approach(p, px, py, tx, ty, s_guess, window=0.25):
    """Arc length s*, distance d* and wire height z* of the closest approach.

    Golden-section search on the squared distance over [s_guess - window,
    s_guess + window] followed by Newton steps on its derivative (analytic
    first and second derivatives of the helix).
    """
    kappa = p[2]

    def f(s):
        return helix_line_distance(p, s, px, py, tx, ty)[0] ** 2

    a, b = max(0.0, s_guess - window), s_guess + window
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(120):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
        if b - a < 1e-13:
            break
    s = 0.5 * (a + b)
    for _ in range(8):
        (gx, gy, gz), (wx, wy, wz), gw = _line_terms(p, s, px, py, tx, ty)
        T = helix_tangent(p, s)
        th = p[1] + kappa * s
        A2 = (-kappa * math.sin(th), kappa * math.cos(th), 0.0)
        Tw = T[0] * wx + T[1] * wy + T[2] * wz
        A2w = A2[0] * wx + A2[1] * wy
        d1 = 2.0 * (gx * T[0] + gy * T[1] + gz * T[2]) - 2.0 * gw * Tw
        d2 = (2.0 * (T[0] ** 2 + T[1] ** 2 + T[2] ** 2 + gx * A2[0] + gy * A2[1])
              - 2.0 * (Tw * Tw + gw * A2w))
        if d2 <= 0.0:
            break
        step = d1 / d2
        s -= step
        if abs(step) < 1e-16:
            break
    dist, zw = helix_line_distance(p, s, px, py, tx, ty)
    return s, dist, zw


# --------------------------------------------------------------------------
# truth helices and events
# --------------------------------------------------------------------------
def draw_helix(rng, chamber=CHAMBER, pt_range=(0.5, 2.0), d0_sigma=1e-3, d0_clip=4.5e-3,
               z0_sigma=1e-2, z0_clip=4.5e-2, tanl_range=(-0.8, 0.8)):
    pt = rng.uniform(*pt_range)
    q = 1.0 if rng.uniform() < 0.5 else -1.0
    kappa = -q * C_LIGHT * chamber.b_field / pt
    phi0 = rng.uniform(0.0, 2.0 * np.pi)
    tanl = rng.uniform(*tanl_range)
    d0 = float(np.clip(rng.normal(0.0, d0_sigma), -d0_clip, d0_clip))
    z0 = float(np.clip(rng.normal(0.0, z0_sigma), -z0_clip, z0_clip))
    return np.array([d0, phi0, kappa, z0, tanl])


def layer_candidates(p, layer, chamber=CHAMBER, n_near=2):
    """(wire index, s*, d*, z*) for the wires of `layer` nearest the helix crossing."""
    r = float(chamber.radius(layer))
    s_c = crossing_arc(p, r)
    if not np.isfinite(s_c):
        return []
    x, y, z = helix_point(p, s_c)
    nw = int(chamber.n_wires(layer))
    tt = float(chamber.tan_tau(layer))
    # azimuth of wire j at height z is about phi_w + z tan(tau) / r
    phc = math.atan2(y, x) - z * tt / r
    j0 = int(round(phc * nw / (2.0 * np.pi) - 0.5 * (layer % 2)))
    out = []
    for dj in range(-n_near, n_near + 1):
        j = (j0 + dj) % nw
        px, py, tx, ty = (float(v) for v in chamber.wire_geometry(layer, j))
        s, d, zw = closest_approach(p, px, py, tx, ty, s_c)
        out.append((j, s, d, zw))
    out.sort(key=lambda t: t[2])
    return out


def helix_hits(p, chamber=CHAMBER, second=False):
    """One hit per layer: the wire closest to the helix (optionally also the 2nd closest)."""
    hits = []
    for layer in range(chamber.n_layers):
        cands = layer_candidates(p, layer, chamber)
        cands = [c for c in cands if abs(c[3]) <= chamber.half_length]
        if not cands:
            continue
        picks = cands[:2] if second else cands[:1]
        for rank, (j, s, d, zw) in enumerate(picks):
            hits.append((layer, j, d, s, zw, rank))
    return hits


# --------------------------------------------------------------------------
# vectorised closest approach: all layers and candidate wires of a helix
# --------------------------------------------------------------------------
def _xyz(p, s):
    d0, phi0, kappa, z0, tanl = p
    R = 1.0 / kappa
    th = phi0 + kappa * s
    return (-(R + d0) * np.sin(phi0) + R * np.sin(th), (R + d0) * np.cos(phi0) - R * np.cos(th),
            z0 + tanl * s)


def crossing_arcs(p, radii):
    """Smallest s > 0 reaching each radius (NaN if never); bisection, 200 steps."""
    radii = np.asarray(radii, dtype=float)
    R = 1.0 / p[2]
    s_hi = np.full(radii.shape, np.pi * abs(R))
    x, y, _ = _xyz(p, s_hi)
    ok = (np.hypot(x, y) >= radii) & (abs(p[0]) <= radii)
    lo, hi = np.zeros(radii.shape), s_hi.copy()
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        x, y, _ = _xyz(p, mid)
        inside = np.hypot(x, y) < radii
        lo = np.where(inside, mid, lo)
        hi = np.where(inside, hi, mid)
    return np.where(ok, 0.5 * (lo + hi), np.nan)


def _perp(p, s, px, py, tx, ty):
    x, y, z = _xyz(p, s)
    n = np.sqrt(tx * tx + ty * ty + 1.0)
    wx, wy, wz = tx / n, ty / n, 1.0 / n
    gx, gy, gz = x - px, y - py, z
    gw = gx * wx + gy * wy + gz * wz
    qx, qy, qz = gx - gw * wx, gy - gw * wy, gz - gw * wz
    return np.sqrt(qx * qx + qy * qy + qz * qz), gw * wz, (gx, gy, gz), (wx, wy, wz), gw


def closest_approach_vec(p, px, py, tx, ty, s_guess, window=0.25):
    """Vectorised golden-section search (100 steps) on the squared helix-line
    distance over [s_guess - window, s_guess + window], then Newton steps on
    its derivative; returns (s*, d*, wire z*)."""
    kappa = p[2]
    a = np.maximum(0.0, s_guess - window)
    b = s_guess + window
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc = _perp(p, c, px, py, tx, ty)[0] ** 2
    fd = _perp(p, d, px, py, tx, ty)[0] ** 2
    for _ in range(100):
        left = fc < fd                      # the minimum lies in [a, d]
        a, b = np.where(left, a, c), np.where(left, d, b)
        c_new = np.where(left, b - g * (b - a), d)
        d_new = np.where(left, c, a + g * (b - a))
        f_new = _perp(p, np.where(left, c_new, d_new), px, py, tx, ty)[0] ** 2
        fc, fd = np.where(left, f_new, fd), np.where(left, fc, f_new)
        c, d = c_new, d_new
    s = 0.5 * (a + b)
    for _ in range(8):
        _, _, (gx, gy, gz), (wx, wy, wz), gw = _perp(p, s, px, py, tx, ty)
        th = p[1] + kappa * s
        T0, T1, T2 = np.cos(th), np.sin(th), p[4]
        A0, A1 = -kappa * np.sin(th), kappa * np.cos(th)
        Tw = T0 * wx + T1 * wy + T2 * wz
        A2w = A0 * wx + A1 * wy
        d1 = 2.0 * (gx * T0 + gy * T1 + gz * T2) - 2.0 * gw * Tw
        d2 = 2.0 * (T0 * T0 + T1 * T1 + T2 * T2 + gx * A0 + gy * A1) - 2.0 * (Tw * Tw + gw * A2w)
        good = d2 > 0.0
        s = s - np.where(good, d1 / np.where(good, d2, 1.0), 0.0)
    dist, zw = _perp(p, s, px, py, tx, ty)[:2]
    return s, dist, zw


def helix_hits_fast(p, chamber=CHAMBER, second=False, n_near=2):
    """helix_hits with the closest approaches of all layers and candidate
    wires computed together."""
    layers = np.arange(chamber.n_layers)
    r = chamber.radius(layers)
    s_c = crossing_arcs(p, r)
    ok = np.isfinite(s_c)
    if not ok.any():
        return []
    s0 = np.where(ok, s_c, 0.0)
    x, y, z = _xyz(p, s0)
    nw = chamber.n_wires(layers)
    tt = chamber.tan_tau(layers)
    phc = np.arctan2(y, x) - z * tt / r
    j0 = np.round(phc * nw / (2.0 * np.pi) - 0.5 * (layers % 2)).astype(np.int64)
    dj = np.arange(-n_near, n_near + 1)
    k = dj.size
    L = np.repeat(layers, k)
    J = (np.repeat(j0, k) + np.tile(dj, layers.size)) % np.repeat(nw, k)
    px, py, tx, ty = chamber.wire_geometry(L, J)
    s_star, d_star, z_star = closest_approach_vec(p, px, py, tx, ty, np.repeat(s0, k))
    hits = []
    for layer in layers:
        if not ok[layer]:
            continue
        cands = [(int(J[i]), float(s_star[i]), float(d_star[i]), float(z_star[i]))
                 for i in range(layer * k, (layer + 1) * k) if abs(z_star[i]) <= chamber.half_length]
        cands.sort(key=lambda t: t[2])
        picks = cands[:2] if second else cands[:1]
        for rank, (j, s, d, zw) in enumerate(picks):
            hits.append((int(layer), j, d, s, zw, rank))
    return hits


@dataclasses.dataclass
class Event:
    hits: np.ndarray            # HIT_DTYPE, shape (N,)
    truth: np.ndarray           # (n_helix, 5)
    owner: np.ndarray           # (N,) helix index, -1 for noise
    layer: np.ndarray           # (N,)
    wire: np.ndarray            # (N,)
    sigma: float

    @property
    def n_hits(self):
        return int(self.hits.shape[0])


def _fill_hit(chamber, layer, j, drift, band):
    x0, y0, z0, x1, y1, z1 = (float(v) for v in chamber.wire_endpoints(layer, j))
    return (x0, y0, z0, x1, y1, z1, float(drift), float(band))


def make_event(rng, n_helix=1, sigma=0.0, noise_frac=0.0, n_hits=None, chamber=CHAMBER,
               noise_round="sig", n_sigma=3.0):
    """Generate one event.

    sigma       Gaussian smearing of drift radii (clipped to [0, half cell]); 0 = noiseless.
    noise_frac  noise = round(noise_frac * n_signal) when n_hits is None (fixed helix
                content), else noise = round(noise_frac * n_hits) and the signal budget
                n_hits - noise is filled helix-major, inner layer first.
    The tolerance band of every hit is n_sigma * sigma.
    """
    truth = np.array([draw_helix(rng, chamber) for _ in range(n_helix)]).reshape(n_helix, 5)
    band = n_sigma * sigma
    used = {}      # (layer, wire) -> row
    rows, owner, layers, wires = [], [], [], []

    def add(layer, j, drift, own):
        key = (layer, j)
        if key in used:
            k = used[key]
            if drift < rows[k][6]:
                rows[k] = _fill_hit(chamber, layer, j, drift, band)
                owner[k] = own
            return False
        used[key] = len(rows)
        rows.append(_fill_hit(chamber, layer, j, drift, band))
        owner.append(own)
        layers.append(layer)
        wires.append(j)
        return True

    def smear(layer, d):
        if sigma <= 0.0:
            return d
        hc = float(chamber.half_cell(layer))
        return float(np.clip(d + rng.normal(0.0, sigma), 0.0, hc))

    per_helix = [helix_hits_fast(truth[h], chamber, second=n_hits is not None) for h in range(n_helix)]
    if n_hits is None:
        for h in range(n_helix):
            for (layer, j, d, s, zw, rank) in per_helix[h]:
                if rank == 0:
                    add(layer, j, smear(layer, d), h)
        n_noise = int(np.floor(noise_frac * len(rows) + 0.5))
    else:
        n_noise = int(np.floor(noise_frac * n_hits + 0.5))
        budget = n_hits - n_noise
        firsts = [(h, t) for h in range(n_helix) for t in per_helix[h] if t[5] == 0]
        seconds = [(h, t) for h in range(n_helix) for t in per_helix[h] if t[5] == 1]
        for (h, (layer, j, d, s, zw, rank)) in firsts + seconds:
            if len(rows) >= budget:
                break
            add(layer, j, smear(layer, d), h)
        n_noise = n_hits - len(rows)
    # noise hits on distinct wires not already hit
    n_layers = chamber.n_layers
    added = 0
    while added < n_noise:
        layer = int(rng.integers(0, n_layers))
        j = int(rng.integers(0, int(chamber.n_wires(layer))))
        if (layer, j) in used:
            continue
        hc = float(chamber.half_cell(layer))
        add(layer, j, rng.uniform(0.0, hc), -1)
        added += 1
    hits = np.array(rows, dtype=HIT_DTYPE)
    return Event(hits=hits, truth=truth, owner=np.array(owner, dtype=np.int64),
                 layer=np.array(layers, dtype=np.int64), wire=np.array(wires, dtype=np.int64),
                 sigma=float(sigma))


def rng_for(config_id, event_index):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(config_id), int(event_index)])))


# --------------------------------------------------------------------------
# the measured workloads
# --------------------------------------------------------------------------
GRID_RANGE_LO = (-5e-3, 0.0, -0.6, -5e-2, -0.8)
GRID_RANGE_HI = (5e-3, 2.0 * np.pi, 0.6, 5e-2, 0.8)


# the noiseless multi-helix family (config 4's helix counts, exact drifts,
# one hit per layer and helix, no noise hits)
NOISELESS_MULTI = 40


def config_event(config_id, event_index):
    """Event `event_index` of workload `config_id` (1..5, or NOISELESS_MULTI)."""
    rng = rng_for(config_id, event_index)
    if config_id in (1, 3):
        return make_event(rng, n_helix=1, sigma=0.0, noise_frac=0.0)
    if config_id == NOISELESS_MULTI:
        return make_event(rng, n_helix=int(rng.integers(1, 6)), sigma=0.0, noise_frac=0.0)
    if config_id == 2:
        return make_event(rng, n_helix=1, sigma=150e-6, noise_frac=0.2)
    if config_id == 4:
        n_h = int(rng.integers(1, 6))
        f = float(rng.uniform(0.0, 0.3))
        n = int(rng.integers(20, 201))
        return make_event(rng, n_helix=n_h, sigma=150e-6, noise_frac=f, n_hits=n)
    if config_id == 5:
        n_h = int(rng.integers(1, 11))
        f = float(rng.uniform(0.0, 0.4))
        n = int(np.clip(np.floor(np.exp(rng.normal(np.log(120.0), 0.6)) + 0.5), 20, 1000))
        return make_event(rng, n_helix=n_h, sigma=150e-6, noise_frac=f, n_hits=n)
    raise ValueError(f"unknown workload {config_id}")


# --------------------------------------------------------------------------
# search schedules (the keyword arguments of Schedule.make / oracle.make_sched)
# --------------------------------------------------------------------------
# the literal schedule of the configs: 16^5, then 4 levels of the top 32 boxes
# split 4^5 each
TOPK_KW = dict(bins=[16] * 5, n_refine=4, top_k=32, split=[4] * 5)
# the window schedule (Sec. 3.3 re-gridding from all max-vote boxes): level 0
# the 16^5 grid over the range, level 1 a 16^5 window, then the reference
# point moves to the hit closest to the recovered circle and six 12^5
# windows follow; the forward-hit test applies before the move, each level
# votes with the hits the previous level's hit finding selected, and every
# level keeps to circles passing within 5 mm of the origin (Eq. ApoVoteDisk);
# windows cover the boxes within one vote of the maximum
WINDOW_LBINS = [[16] * 5, [16] * 5] + [[12] * 5] * 6
WINDOW_KW = dict(bins=[16] * 5, n_refine=7, mode=1, forward=True, move_level=1, lbins=WINDOW_LBINS, hitsel=True,
                 disk=5e-3, wdrop=1)
# the recovery tolerances on (d0, phi0, kappa, z0, tanl)
RECOVERY_TOL = (1e-3, 5e-3, 0.01, 10e-3, 0.02)
# the transverse part of them alone (z0 and tanl free)
TRANSVERSE_TOL = (1e-3, 5e-3, 0.01, np.inf, np.inf)


def match_helices(found, truth, tol=RECOVERY_TOL):
    """For each found helix (rows of p), the index of the first generated
    helix it recovers, or -1."""
    out = []
    for p in found:
        m = -1
        for t in range(len(truth)):
            if recovered(p, truth[t], tol):
                m = t
                break
        out.append(m)
    return np.array(out, dtype=np.int64)


def recovered(p, truth, tol=RECOVERY_TOL):
    """p within tol of truth in every parameter (phi0 compared on the circle)."""
    d = np.abs(np.asarray(p, dtype=float) - np.asarray(truth, dtype=float))
    d[1] = d[1] % (2.0 * np.pi)
    d[1] = min(d[1], 2.0 * np.pi - d[1])
    return bool(np.all(d <= np.asarray(tol)))
