// ia_kernels.hpp -- HIP kernels of the interval-arithmetic helix vote (gfx950).
//
// Box order everywhere: a level is n_parents parent boxes, each split
// regularly by m[5] (dimension order d0, phi0, kappa, z0, tanl; d0 slowest,
// tanl fastest); box b = parent * prod(m) + child.  Child edges are
// L + k (U - L)/m, the last edge U (Sec. 3.3 voxel grids).
//
// The vote of a hit for a box depends on the box's (d0, phi0, kappa)
// intervals -- a "triple" -- through the interval residual G, and on its
// (z0, tanl) centre only through the point-evaluated stereo drift d^Ax.  The
// vote kernel therefore stages, per (triple, hit), everything that does not
// depend on (z0, tanl) in LDS (computed cooperatively by the workgroup), and
// each lane (one box) finishes the stereo term for its own (z0, tanl).  Axial
// hits (tan tau = 0) are decided completely per (triple, hit).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ia_math.hpp"

namespace ia {

constexpr int kWG = 256;        // lanes per workgroup (4 waves of 64)
constexpr int kCap = 256;       // (triple, hit) records staged per chunk
constexpr int kHistLds = 1024;  // vote histogram bins kept in LDS
constexpr int kHistLdsRec = 512; // the same in k_vote_rec, whose staged records take more LDS
constexpr int kEstLevels = 15;  // estimate stack depth (partials of up to 2^22 boxes)
constexpr int kMaxTopK = 4096;  // selection size limit

struct HitRec {                 // prepared hit, 112 bytes
  double px, py, tant, sphis, cphis, r, phip, r2lo, r2hi, d, band;
  double sphp, cphp;            // sin and cos of phip (sin_p, cos_p)
  int32_t use;                  // 0: not searched (malformed or assigned); bit 0: active in the
                                // pass (a hit-finding candidate); 1: also votes at this level,
                                // 3: not selected to vote at this level
  int32_t axial;
};

// the hit votes at the current level
IA_HD bool votes_now(const HitRec& h) { return h.use == 1; }

struct BoxD { double lo[5], hi[5]; };

struct Shape {                  // one level of boxes (n_boxes < 2^31)
  uint32_t m[5];
  uint32_t nc;                  // boxes per parent
  uint32_t m34;                 // (z0, tanl) boxes per triple
  uint32_t m012;                // triples per parent
  uint32_t m12;                 // m[1] * m[2]
  uint32_t n_boxes;             // n_parents * nc
  uint32_t n_parents;
  uint32_t pad;
};

// per-event control block kept on the device
struct EventState {
  int32_t done;                 // 1: no further work for this event
  int32_t n_out;                // helices written
  int32_t vmax;                 // max votes of the last selection
  int32_t k_sel;                // boxes selected by the last selection
  int32_t n_assigned;           // hits assigned by the last hit finding
  int32_t n_argmax;             // size of the max-vote set of the last level
  int32_t t_prune;              // vote threshold of the current level's pruning (0: none)
  int32_t n_live;               // vote tiles of the current level holding a box that can be selected
  int32_t n_live_tri;           // triples of the current level whose class-2 pairs are evaluated
  int32_t n_rec;                // their class-2 pairs (staged records)
  int32_t rec_ok;               // 1: the records fit the record buffer (else the in-kernel staging runs)
  int32_t t_cut;                // triples after this one with upper bound == t_prune are pruned too
  int32_t moving;               // window schedule: 1 while the reference point is being moved
  int32_t moved;                // window schedule: 1 once it moved in this pass
  double p[5], err[5];          // last estimate
  double ulo[5], uhi[5];        // union of the last level's max-vote boxes (phi0 relative to the first)
  double ref[2];                // reference point of the current level (origin coordinates)
  double shift[2];              // move of the reference point under way (the chosen hit point)
  uint32_t occ[32];             // window schedule: phi0 bins holding max-vote boxes (bit mask)
  int32_t run_a, run_b;         // their run holding the first max-vote box (run_a < 0: all bins)
};

constexpr uint32_t kRunMaxBins = 1024;   // phi0 bins the run selection handles

// phi0 bin of box b of a level
IA_HD uint32_t phi_bin(const Shape& sh, uint32_t b) {
  return ((b % sh.nc) / (sh.m[2] * sh.m[3] * sh.m[4])) % sh.m[1];
}

IA_HD bool in_run(uint32_t k, int32_t a, int32_t b) {
  if (a < 0) return true;
  const int32_t kk = static_cast<int32_t>(k);
  return a <= b ? (kk >= a && kk <= b) : (kk >= a || kk <= b);
}

// Per-event views of a batch of events launched together: blockIdx.y is the
// event.  Event e owns hits [off[e], off[e+1]) of the prepared-hit array
// (off == nullptr: one event of n_single hits) and the e-th slice of every
// per-event array, at the strides below.
struct EvView {
  const int32_t* off;
  int32_t n_single;
  int32_t k;                    // selection size (stride of the selection arrays)
  int64_t par_stride;           // parent boxes per event (0: one shared list)
  int64_t flag_stride;          // pre-pass flags per event
  int64_t tri_stride;           // per-triple vote bounds per event
  int64_t rec_stride;           // staged pair records per event
  int64_t pflag_stride;         // parent-level exclusion flags per event
  int32_t hist_stride;          // histogram bins per event
  int32_t wg_stride;            // workgroup maxima per event
  int32_t part_stride;          // estimate chunk sums per event (doubles)
  int32_t max_out;              // helices per event
  int32_t max_hits;             // hits per event the strides are sized for (0: unchecked)
  int64_t n_total;              // hits addressable from the batch's first hit
  int32_t fwd;                  // 1: forward-hit test at this level
  double disk;                  // disk condition radius (0: off)
  double vref[2];               // reference point of the level when there is no event state
  const int32_t* cnt;           // hits per event when events sit in fixed-size rows (off[e] the row start)
  __device__ int32_t beg(int e) const { return off ? off[e] : 0; }
  __device__ int32_t count(int e) const { return cnt ? cnt[e] : (off ? off[e + 1] - off[e] : n_single); }
};

// status word bits (device-detected problems, read after a stream sync)
enum : uint32_t { kStBadHit = 1u, kStVoteOverflow = 2u, kStBadOffsets = 4u };

// work counters: kWorkSlots slots of 16 u64 (one 128-byte line each);
// counters 0..3 of a slot: stereo (box, hit) evaluations and staged (triple,
// hit) pairs at FP64 levels, the same two at FP32 levels (vote kernels);
// counters kWorkClassify + kCwN p + c: classification work at precision p
// (0 FP64, 1 FP32), c = kCw* below (the first four from k_classify, the
// last three from k_classify_defer)
constexpr uint32_t kWorkSlots = 64;
constexpr uint32_t kWorkSlotU64 = 32;
constexpr uint32_t kWorkClassify = 4;
enum : uint32_t {
  kCwG = 0, kCwAxial = 1, kCwGExact = 2, kCwPairQ = 3, kCwMag = 4,    // first stage
  kCwDefer = 5, kCwPass = 6, kCwIncl = 7,                              // second stage
  kCwN = 8
};
// class flags of a stereo pair whose class k_classify left to
// k_classify_defer: kFlagDeferred with both drift signs open, + 1 with only
// dS = +d open, + 2 with only dS = -d open (the other sign casts no vote in
// any box of the triple)
constexpr uint8_t kFlagDeferred = 3;
// drift signs (bit 0: +d, bit 1: -d) of a deferred flag, and the flag of a set
IA_HD int defer_signs(uint8_t fl) { return fl == kFlagDeferred ? 3 : fl - kFlagDeferred; }
IA_HD uint8_t defer_flag(int signs) { return static_cast<uint8_t>(signs == 3 ? kFlagDeferred : kFlagDeferred + signs); }

// ---------------------------------------------------------------------------
// edges of child k of [L, U] split m ways
IA_HD void child_edge(double L, double U, uint32_t m, uint32_t k,
                                           double* lo, double* hi) {
  double w = (U - L) / static_cast<double>(m);
  *lo = L + static_cast<double>(k) * w;
  *hi = (k + 1 == m) ? U : L + static_cast<double>(k + 1) * w;
}

IA_HD void child_index(const uint32_t m[5], uint32_t child, uint32_t k[5]) {
  for (int j = 4; j >= 0; --j) { k[j] = child % m[j]; child /= m[j]; }
}

IA_HD void child_box(const BoxD& P, const uint32_t m[5], uint32_t child, BoxD* out) {
  uint32_t k[5];
  child_index(m, child, k);
  for (int j = 0; j < 5; ++j) child_edge(P.lo[j], P.hi[j], m[j], k[j], &out->lo[j], &out->hi[j]);
}

IA_HD void level_box(const BoxD* parents, const Shape& sh, uint32_t b, BoxD* out) {
  child_box(parents[b / sh.nc], sh.m, b % sh.nc, out);
}

// ---------------------------------------------------------------------------
// hit preparation (Eqs. wirePar_a,b and EQSinter_d,e with z_ref = 0)
// The hit point is taken about the reference point (xr, yr) of the level's
// parametrisation: the wire point at z = 0 less (xr, yr), one rounding each
// (exact for the origin).
IA_HD void prep_one(const double* h, bool active, HitRec* o, bool* bad, double xr = 0.0, double yr = 0.0) {
  HitRec r{};
  bool fin = true;
  for (int i = 0; i < 8; ++i) fin = fin && __builtin_isfinite(h[i]);
  *bad = false;
  r.use = 0;
  r.axial = 0;
  if (!fin) { *bad = true; *o = r; return; }
  double x0 = h[0], y0 = h[1], z0 = h[2], x1 = h[3], y1 = h[4], z1 = h[5];
  double dz = z1 - z0;
  if (dz == 0.0 || h[6] < 0.0 || h[7] < 0.0) { *bad = true; *o = r; return; }
  double tx = (x1 - x0) / dz, ty = (y1 - y0) / dz;
  r.px = (x0 - z0 * tx) - xr;
  r.py = (y0 - z0 * ty) - yr;
  r.tant = sqrt(tx * tx + ty * ty);
  if (!__builtin_isfinite(r.px) || !__builtin_isfinite(r.py) || !__builtin_isfinite(r.tant)) { *bad = true; *o = HitRec{}; return; }
  if (r.tant == 0.0) { r.sphis = 0.0; r.cphis = 1.0; r.axial = 1; }
  else { r.sphis = tx / r.tant; r.cphis = -ty / r.tant; r.axial = 0; }
  r.r = sqrt(r.px * r.px + r.py * r.py);
  r.phip = atan2_p(r.py, r.px);
  r.sphp = sin_p(r.phip);
  r.cphp = cos_p(r.phip);
  double r2 = r.r * r.r;
  r.r2lo = wdn(r2);
  r.r2hi = wup(r2);
  r.d = h[6];
  r.band = h[7];
  r.use = active ? 1 : 0;
  *o = r;
}

// ---------------------------------------------------------------------------
// frame of a triple at its centre (mirrored to kappa > 0, Appendix A assumes R > 0)
struct Frame {
  Iv K, Dd, Fi;                 // kappa, d0, phi0 intervals
  double sig, R, xc, yc, sp0, cp0;
};

IA_HD Frame triple_frame(const BoxD& P, const uint32_t m[5], uint32_t k0, uint32_t k1,
                                              uint32_t k2) {
  Frame f;
  child_edge(P.lo[0], P.hi[0], m[0], k0, &f.Dd.lo, &f.Dd.hi);
  child_edge(P.lo[1], P.hi[1], m[1], k1, &f.Fi.lo, &f.Fi.hi);
  child_edge(P.lo[2], P.hi[2], m[2], k2, &f.K.lo, &f.K.hi);
  double c0 = 0.5 * (f.Dd.lo + f.Dd.hi), c1 = 0.5 * (f.Fi.lo + f.Fi.hi), kap = 0.5 * (f.K.lo + f.K.hi);
  double sig = 1.0;
  if (kap < 0.0) sig = -1.0;
  if (kap == 0.0) { kap = 0x1p-30; sig = 1.0; }
  double kp = sig * kap, d0p = sig * c0;
  double s1, c1v;
  s1 = sin_p(c1);
  c1v = cos_p(c1);
  f.sp0 = sig * s1;
  f.cp0 = c1v;
  f.R = 1.0 / kp;
  double Rd = f.R + d0p;
  f.xc = -(Rd * f.sp0);
  f.yc = Rd * f.cp0;
  f.sig = sig;
  return f;
}

// interval residual G over the triple (kappa-scaled Eq. ApoVote)
IA_HD Iv residual_G(const Frame& f, const HitRec& h) {
  Iv Ar = {wdn(f.Fi.lo - h.phip), wup(f.Fi.hi - h.phip)};
  Iv S = sin_encl(Ar.lo, Ar.hi);
  Iv rS = imul_pos(S, h.r);
  Iv D2 = isqr(f.Dd);
  Iv T0 = iadd(D2, Iv{h.r2lo, h.r2hi});
  Iv T = {0.5 * T0.lo, 0.5 * T0.hi};
  Iv KT = imul(f.K, T);
  Iv KD1 = iadd(imul(f.K, f.Dd), Iv{1.0, 1.0});
  return iadd(iadd(KT, imul(KD1, rS)), f.Dd);
}

// Forward-hit test over the phi0 interval of a triple: the hit point is ahead
// of the point of closest approach for some phi0 when the enclosure of
// cos(phi0 - phiP) = sin(phi0 - phiP + pi/2) reaches above zero (pi/2 taken
// below it at the lower end, above it at the upper end, the ends rounded
// outward).  A hit at the reference point is ahead.
IA_HD bool forward_ok(const Iv& Fi, const HitRec& h) {
  if (h.r == 0.0) return true;
  const Iv S = sin_encl(wdn(wdn(Fi.lo - h.phip) + kPio2), wup(wup(Fi.hi - h.phip) + kPio2Up));
  return S.hi > 0.0;
}

// Direction test about a moved reference point (xr, yr): for some phi0 of the
// triple the origin, seen from the point of closest approach, lies behind it
// (the track comes from the origin): the enclosure of cos(phi0 - phi_O) =
// sin(phi0 - phi_O + pi/2) reaches below zero, phi_O the direction of the
// origin from the reference point.
IA_HD bool behind_ok(const Iv& Fi, double xr, double yr) {
  if (xr == 0.0 && yr == 0.0) return true;
  const double phio = atan2_p(-yr, -xr);
  const Iv S = sin_encl(wdn(wdn(Fi.lo - phio) + kPio2), wup(wup(Fi.hi - phio) + kPio2Up));
  return S.lo < 0.0;
}

// Perigee parameters p about a reference point -> q about that point moved by
// (dx, dy).  With n = (-sin phi0, cos phi0) and u = (cos phi0, sin phi0),
// A = (1 + kappa d0) n - kappa D is kappa times the vector from the new point
// to the circle's centre, so phi0' = atan2(-A_x, A_y) and
// d0' = (2 d0 + kappa d0^2 - 2 (1 + kappa d0) n.D + kappa |D|^2) / (|A| + 1),
// finite for kappa -> 0; the direction turns by
// atan2(kappa u.D, 1 + kappa d0 - kappa n.D) over the arc s between the two
// points of closest approach (s = u.D for kappa = 0), and z0' = z0 + tanl s.
// the transverse part: d0', phi0' and the arc between the two points of
// closest approach
IA_HD void frame_shift_t(double d0, double f0, double k, double dx, double dy, double* d1, double* f1o,
                         double* arc_o) {
  const double s0 = sin_p(f0), c0 = cos_p(f0);
  const double nD = -s0 * dx + c0 * dy;
  const double uD = c0 * dx + s0 * dy;
  const double one = 1.0 + k * d0;
  const double ax = one * (-s0) - k * dx;
  const double ay = one * c0 - k * dy;
  const double A = sqrt(ax * ax + ay * ay);
  const double num = 2.0 * d0 + k * (d0 * d0) - 2.0 * one * nD + k * (dx * dx + dy * dy);
  double f1 = atan2_p(-ax, ay);
  if (f1 < 0.0) f1 += kTwoPi;
  double arc = uD;
  if (k != 0.0) arc = atan2_p(k * uD, one - k * nD) / k;
  *d1 = num / (A + 1.0);
  *f1o = f1;
  *arc_o = arc;
}

IA_HD void frame_shift(const double* p, double dx, double dy, double* q) {
  double arc;
  frame_shift_t(p[0], p[1], p[2], dx, dy, &q[0], &q[1], &arc);
  q[2] = p[2];
  q[3] = p[3] + p[4] * arc;
  q[4] = p[4];
}

// The disk condition (Eq. ApoVoteDisk): some circle of the triple passes
// within `disk` of the origin.  It is Eq. ApoVote for a measurement at the
// origin with drift 0 and tolerance `disk`: an axial hit whose point is the
// origin taken about the reference point (xr, yr).
IA_HD HitRec disk_hit(double xr, double yr, double disk) {
  HitRec h{};
  h.px = -xr;
  h.py = -yr;
  h.tant = 0.0;
  h.sphis = 0.0;
  h.cphis = 1.0;
  h.r = sqrt(h.px * h.px + h.py * h.py);
  h.phip = h.r == 0.0 ? 0.0 : atan2_p(h.py, h.px);
  const double r2 = h.r * h.r;
  h.r2lo = wdn(r2);
  h.r2hi = wup(r2);
  h.d = 0.0;
  h.band = disk;
  h.use = 1;
  h.axial = 1;
  return h;
}

// G of the kappa-scaled Eq. ApoVote at one parameter point: to first order
// the distance of the hit point from the circle
IA_HD double point_G(const HitRec& h, const double* p) {
  const double d0 = p[0], k = p[2];
  return 0.5 * k * (h.r * h.r + d0 * d0) + (1.0 + k * d0) * (h.r * sin_p(p[1] - h.phip)) + d0;
}

// An outer enclosure of residual_G for exclusion tests, cheaper per pair.
// residual_G's operations are kept except the sin enclosure S of
// [phi0 - phip], which is replaced by an interval holding it: the sines at the
// two ends come from the difference identity with the triple's sin / cos of
// its phi0 edges and the hit's sin / cos of phip (each within 0.56 ulp), so
// they lie within a few ulps of sin_p at those ends, and a margin of 2^-46
// covers that, sin_encl's 2^-50 and the one-ulp widening of the angles; an
// extremum is taken as soon as the cosines at the ends change sign within
// 1e-6 (the phi0 range is narrower than pi, else [-1, 1]).  Every later
// operation is inclusion-monotone, so the result holds residual_G's: an H
// test failing for it fails for residual_G too.  GTri holds the per-triple
// parts.
struct GTri {
  Iv D2, KD1;
  double sa, ca, sb, cb;        // sin, cos of the phi0 edges
  int32_t wide;
};

IA_HD GTri g_triple(const Frame& f) {
  GTri g;
  g.D2 = isqr(f.Dd);
  g.KD1 = iadd(imul(f.K, f.Dd), Iv{1.0, 1.0});
  g.sa = sin_p(f.Fi.lo);
  g.ca = cos_p(f.Fi.lo);
  g.sb = sin_p(f.Fi.hi);
  g.cb = cos_p(f.Fi.hi);
  g.wide = !(f.Fi.hi - f.Fi.lo <= 3.0);
  return g;
}

IA_HD Iv residual_G_outer(const Frame& f, const GTri& g, const HitRec& h) {
  constexpr double mS = 0x1p-46, mC = 1e-6;
  Iv S = {-1.0, 1.0};
  if (!g.wide) {
    const double s_a = g.sa * h.cphp - g.ca * h.sphp, s_b = g.sb * h.cphp - g.cb * h.sphp;
    const double c_a = g.ca * h.cphp + g.sa * h.sphp, c_b = g.cb * h.cphp + g.sb * h.sphp;
    const bool has_max = c_a >= -mC && c_b <= mC;
    const bool has_min = c_a <= mC && c_b >= -mC;
    S.hi = has_max ? 1.0 : fmin(1.0, fmax(s_a, s_b) + mS);
    S.lo = has_min ? -1.0 : fmax(-1.0, fmin(s_a, s_b) - mS);
  }
  const Iv rS = imul_pos(S, h.r);
  const Iv T0 = iadd(g.D2, Iv{h.r2lo, h.r2hi});
  const Iv T = {0.5 * T0.lo, 0.5 * T0.hi};
  const Iv KT = imul(f.K, T);
  return iadd(iadd(KT, imul(g.KD1, rS)), f.Dd);
}

IA_HD bool h_contains0(Iv G, Iv K, double e, double band) {
  Iv E = {wdn(e - band), wup(e + band)};
  Iv Hv = isub(itwice(G), iadd(itwice(E), imul(K, isqr(E))));
  return (Hv.lo <= 0.0) & (0.0 <= Hv.hi);
}

// h_contains0 with the same result in fewer operations, for the branch-free
// per-box evaluation.  With S = E^2 and S.lo >= 0 (otherwise *ok is
// cleared), the smallest of the four products K x S is K.lo S.lo for
// K.lo >= 0 and K.lo S.hi otherwise, and the largest K.hi S.hi for
// K.hi >= 0 and K.hi S.lo otherwise (rounding to nearest is monotone), so
// two products give imul's end points.  The last outward roundings are
// folded into the comparisons: wdn(x) <= 0 exactly when x <= 2^-1074, and
// wup(x) >= 0 exactly when x >= -2^-1074.  *sq_ok tells whether S.lo >= 0
// held (the result stands only then).
IA_HD bool h_contains0_fast(Iv G, Iv K, double e, double band, bool* sq_ok) {
  const Iv E = {wdn(e - band), wup(e + band)};
  const Iv S = isqr(E);
  *sq_ok = S.lo >= 0.0;
  const Iv KS = {wdn(K.lo * (K.lo >= 0.0 ? S.lo : S.hi)), wup(K.hi * (K.hi >= 0.0 ? S.hi : S.lo))};
  const Iv T = iadd(itwice(E), KS);
  const double lo = 2.0 * G.lo - T.hi, hi = 2.0 * G.hi - T.lo;
  return (lo <= 0x1p-1074) & (hi >= -0x1p-1074);
}

// per (triple, stereo hit) quantities that do not depend on (z0, tanl)
struct PairQ {
  double Glo, Ghi, sArc, dphi, RAx, sinA, cosA, sAx, cAx, c2, s2, twoRAx2, RpRAx;
  // recip_v of RAx and of twoRAx2 (the per-box quotients' divisors); r2RAx2
  // is NaN too when the drift is outside [2^-200, 2^200] (drift_ok), so that
  // the branch-free per-box form, which divides by the drift's range, is
  // left for the plain one
  double rRAx, r2RAx2;
};

IA_HD bool drift_ok(double d) { return d >= 0x1p-200 && d <= 0x1p200; }

IA_HD PairQ pair_quantities(const Frame& f, const HitRec& h, Iv G) {
  PairQ q;
  q.Glo = G.lo;
  q.Ghi = G.hi;
  double py = f.sig * h.py, cps = f.sig * h.cphis, sps = h.sphis;
  double Dx = h.px - f.xc, Dy = py - f.yc;
  q.RAx = sqrt(Dx * Dx + Dy * Dy);
  q.cAx = Dx * sps - Dy * cps;
  q.sAx = Dx * cps + Dy * sps;
  q.sinA = q.sAx / q.RAx;
  q.cosA = q.cAx / q.RAx;
  q.dphi = atan2_p(Dx * f.cp0 + Dy * f.sp0, Dx * f.sp0 - Dy * f.cp0);
  q.sArc = f.R * q.dphi;
  q.c2 = q.cosA * q.cosA - q.sinA * q.sinA;
  q.s2 = 2.0 * q.sinA * q.cosA;
  q.twoRAx2 = 2.0 * (q.RAx * q.RAx);
  q.RpRAx = f.R + q.RAx;
  q.rRAx = recip_v(q.RAx);
  q.r2RAx2 = drift_ok(h.d) ? recip_v(q.twoRAx2) : __builtin_nan("");
  return q;
}

// fixed-point steps of Eq. CSAXtoPHI_a at IA_FP64X levels
constexpr int kPhiIters = 3;

// stereo vote of one hit for one box centre (z0, lam); ApproxPhi, normudi,
// EQSinter_c, defdiAX_b evaluated in the same operation order as the oracle.
// EXACT: Phi - Phi^Ax from kPhiIters fixed-point steps of Eq. CSAXtoPHI_a,
// eps <- atan2(s^tau tan(tau), (R^Ax)^2 + c^tau tan(tau)), started from ApproxPhi.
//
// FAST (device only): the same operations with three primitives replaced by
// forms that give the same bits on a stated range (ia_math.hpp): the two
// quotients by per-pair divisors (div_fast, reciprocals staged in PairQ),
// the square roots (sqrt_fast) and sin/cos of the correction without the
// range reduction.  It has no branches, so the two drift signs interleave;
// each replaced step clears *ok when its input is outside its range, and the
// caller then evaluates the box again in the plain form.
template <bool EXACT, bool FAST>
IA_HD bool stereo_vote_t(const PairQ& q, double R, double sig, Iv K, double z0, double lam, double lamR,
                         double lam2, double tt, double t2, double d, double band, bool* ok) {
  double zA = z0 + lam * q.sArc;
  double zAs = zA * q.sinA;
  double zA2 = zA * zA;
  double lzA = lam * zA;
  Iv G = {q.Glo, q.Ghi};
  bool vote = false;
#pragma unroll
  for (int si = 0; si < 2; ++si) {
    double dS = si == 0 ? d : -d;
    double Phi1, Phi2;
    const double Phi2n =
        lamR * zA - (lzA * (R - 2.0 * dS)) * q.c2 + (zA2 + dS * (q.RAx + lam2 * (q.RpRAx - dS))) * q.s2;
    if constexpr (FAST) {
      Phi1 = div_fast(-(zAs + (lam * dS) * q.cosA), q.RAx, q.rRAx, ok);
      Phi2 = div_fast(Phi2n, q.twoRAx2, q.r2RAx2, ok);
    } else {
      Phi1 = -(zAs + (lam * dS) * q.cosA) / q.RAx;
      Phi2 = Phi2n / q.twoRAx2;
    }
    double eps = Phi1 * tt + Phi2 * t2;
    if constexpr (EXACT) {
      const double RAx2 = q.RAx * q.RAx;
      for (int it = 0; it < kPhiIters; ++it) {
        double s1, c1;
        sincos_p(eps, &s1, &c1);
        const double sP = q.sinA * c1 + q.cosA * s1, cP = q.cosA * c1 - q.sinA * s1;
        const double uu = sqrt(((1.0 + ((2.0 * lam) * sP) * tt) + lam2 * t2) + (cP * cP) * t2);
        const double dl = dS / uu;
        const double sp = R * (q.dphi + eps);
        const double zz = (z0 + lam * sp) - (dl * cP) * tt;
        const double l_d = lam * dl;
        const double ct = zz * q.cAx - l_d * q.sAx;
        const double st = -(l_d * q.cAx + zz * q.sAx);
        eps = atan2_p(st * tt, RAx2 + ct * tt);
      }
    }
    double se, ce;
    if constexpr (FAST) {
      // |eps| < pi/4: the reduction of sincos_p is the identity
      const double aeps = fabs(eps);
      *ok = *ok & (aeps < kPio4);
      se = poly_sin(eps);
      ce = poly_cos(eps);
    } else {
      sincos_p(eps, &se, &ce);
    }
    double sinP = q.sinA * ce + q.cosA * se, cosP = q.cosA * ce - q.sinA * se;
    const double u2 = ((1.0 + ((2.0 * lam) * sinP) * tt) + lam2 * t2) + (cosP * cosP) * t2;
    double u, delta;
    if constexpr (FAST) {
      // u in [2^-300, 2^300] and |dS| in [2^-200, 2^200] (the record's
      // r2RAx2 is NaN otherwise, which failed the Phi2 check): the quotient's
      // range holds, so div_exact gives dS / u
      u = sqrt_fast(u2, ok, 0x1p-600, 0x1p600);
      delta = div_exact(dS, u, rcp_newton(u));
    } else {
      u = sqrt(u2);
      delta = dS / u;
    }
    double sperp = R * (q.dphi + eps);
    double zS = (z0 + lam * sperp) - (delta * cosP) * tt;
    double ld = lam * delta;
    double ctau = zS * q.cAx - ld * q.sAx;
    double a1 = zS * tt, a2 = ld * tt;
    double Q = ((2.0 * ctau) * tt + a1 * a1) + a2 * a2;
    double A = R + delta;
    double disc = A * A - Q;
    if constexpr (FAST) {
      // a negative (or NaN) discriminant casts no vote whatever its root
      bool ok_d = true;
      const double dhat = delta - Q / (A + sqrt_fast(disc, &ok_d));
      *ok = *ok & (ok_d | !(disc >= 0.0));
      const double e = sig * dhat;
      bool sq_ok;
      const bool fin = __builtin_isfinite(e), hit = h_contains0_fast(G, K, e, band, &sq_ok);
      const bool used = (disc >= 0.0) & fin;   // the H test decides only then
      *ok = *ok & (sq_ok | !used);
      vote = vote | (used & hit);
    } else if (disc >= 0.0) {
      double dhat = delta - Q / (A + sqrt(disc));
      double e = sig * dhat;
      if (__builtin_isfinite(e) && h_contains0(G, K, e, band)) vote = true;
    }
  }
  return vote;
}

template <bool EXACT = false>
IA_HD bool stereo_vote(const PairQ& q, double R, double sig, Iv K, double z0, double lam, double lamR,
                       double lam2, double tt, double t2, double d, double band) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (!EXACT) {
    bool ok = true;
    const bool v = stereo_vote_t<false, true>(q, R, sig, K, z0, lam, lamR, lam2, tt, t2, d, band, &ok);
    if (ok) return v;
  }
#endif
  return stereo_vote_t<EXACT, false>(q, R, sig, K, z0, lam, lamR, lam2, tt, t2, d, band, nullptr);
}

// ---------------------------------------------------------------------------
// Pre-filter of a (triple, stereo hit) pair.  The point value e of each box
// depends on the box only through its (z0, tanl) centre.  e_enclosure runs
// the operation sequence of stereo_vote in interval arithmetic over the
// rectangle Z x L holding every centre of the triple's boxes, and widens the
// result by 1e-9 |e| + 1e-12 m, far above the rounding error of the point
// evaluation (about 100 ulps of the terms of d^Ax).  Every interval
// operation is inclusion-monotone, so if the H test fails for the widened
// enclosure it fails for every box: the pair casts no vote anywhere in the
// triple.  Returns false when no finite enclosure is available.
IA_HD bool e_enclosure_dom(const PairQ& q, double R, double sig, double tt, double t2, Iv DS, Iv Z, Iv L,
                           Iv* out, Iv* eps_out, Iv* disc_out, Iv* a_out) {
  const Iv ZA = iadd(Z, imul_pt(L, q.sArc));
  const Iv ZAs = imul_pt(ZA, q.sinA);
  const Iv ZA2 = isqr(ZA);
  const Iv LZA = imul(L, ZA);
  const Iv LR = imul_pt(L, R);
  const Iv L2 = isqr(L);
  const Iv PHI1 = ineg(idivp(iadd(ZAs, imul_pt(imul(L, DS), q.cosA)), q.RAx));
  const Iv P2a = imul(LR, ZA);
  const Iv P2b = imul_pt(imul(LZA, isub(ipt(R), itwice(DS))), q.c2);
  const Iv inner = iadd(ipt(q.RAx), imul(L2, isub(ipt(q.RpRAx), DS)));
  const Iv P2c = imul_pt(iadd(ZA2, imul(DS, inner)), q.s2);
  const Iv PHI2 = idivp(iadd(isub(P2a, P2b), P2c), q.twoRAx2);
  const Iv EPS = iadd(imul_pt(PHI1, tt), imul_pt(PHI2, t2));
  *eps_out = EPS;
  if (!(fabs(EPS.lo) < 1e5 && fabs(EPS.hi) < 1e5)) return false;
  Iv SE, CE;
  if (fabs(EPS.lo) <= kSmallTrig && fabs(EPS.hi) <= kSmallTrig) {
    sincos_encl_small(EPS, &SE, &CE);
  } else {
    SE = sin_encl(EPS.lo, EPS.hi);
    CE = cos_encl(EPS.lo, EPS.hi);
  }
  const Iv SINP = iadd(imul_pt(CE, q.sinA), imul_pt(SE, q.cosA));
  const Iv COSP = isub(imul_pt(CE, q.cosA), imul_pt(SE, q.sinA));
  const Iv U2 = iadd(iadd(iadd(ipt(1.0), imul_pt(imul(itwice(L), SINP), tt)), imul_pt(L2, t2)),
                     imul_pt(isqr(COSP), t2));
  if (!(U2.lo > 0.0)) return false;
  const Iv DELTA = idiv_pos2(DS, isqrt(U2));
  const Iv SPERP = imul_pt(iadd(ipt(q.dphi), EPS), R);
  const Iv ZS = isub(iadd(Z, imul(L, SPERP)), imul_pt(imul(DELTA, COSP), tt));
  const Iv LD = imul(L, DELTA);
  const Iv CTAU = isub(imul_pt(ZS, q.cAx), imul_pt(LD, q.sAx));
  const Iv Q = iadd(iadd(imul_pt(itwice(CTAU), tt), isqr(imul_pt(ZS, tt))), isqr(imul_pt(LD, tt)));
  const Iv A = iadd(ipt(R), DELTA);
  const Iv DISC = isub(isqr(A), Q);
  *disc_out = DISC;
  *a_out = A;
  if (!(DISC.hi >= 0.0)) return false;
  const Iv DEN = iadd(A, isqrt(DISC));
  if (!(DEN.lo > 0.0)) return false;
  const Iv DHAT = isub(DELTA, idiv_pos2(Q, DEN));
  const Iv E = sig > 0.0 ? DHAT : ineg(DHAT);
  const double m = 1e-9 * fmax(fabs(E.lo), fabs(E.hi)) + 1e-12;
  *out = {wdn(E.lo - m), wup(E.hi + m)};
  return __builtin_isfinite(out->lo) && __builtin_isfinite(out->hi);
}

IA_HD bool e_enclosure(const PairQ& q, double R, double sig, double tt, double t2, double dS, Iv Z, Iv L, Iv* out) {
  Iv eps, disc, a;
  return e_enclosure_dom(q, R, sig, tt, t2, ipt(dS), Z, L, out, &eps, &disc, &a);
}

// The same enclosure in FP32 interval arithmetic (the form the second stage
// of the classification runs).  Every FP64 input enters as an FP32 interval
// holding it (thin32, cover32) and every operation rounds outward, so the
// result still holds the exact d^Ax of the FP64 pair quantities over Z x L,
// and the same margin 1e-9 |e| + 1e-12 m covers the point evaluation's
// rounding; FP32 only makes the enclosure wider, by a few 1e-7 of the terms'
// size.  The inputs are bounded (R <= 2^40, |z0| <= 2^20, |tanl| <= 2^10,
// |tan tau| <= 16, d <= 2^10, finite pair quantities) so that no
// intermediate comes near the FP32 range; outside those bounds, or when
// |eps| may exceed 0.75, no enclosure is returned (the caller then treats
// the pass as undecided).
struct EnclIn32 {
  Iv32 Z, L, sArc, sinA, cosA, RAx, c2, s2, twoRAx2, RpRAx, dphi, cAx, sAx, R, tt, t2, d;
  bool ok;
};

IA_HD EnclIn32 encl_in32(const PairQ& q, double R, double tt, double t2, double d, Iv Z, Iv L) {
  EnclIn32 c;
  const double qs = q.sArc + q.sinA + q.cosA + q.RAx + q.c2 + q.s2 + q.twoRAx2 + q.RpRAx + q.dphi + q.cAx + q.sAx;
  c.ok = R <= 0x1p40 && fmax(fabs(Z.lo), fabs(Z.hi)) <= 0x1p20 && fmax(fabs(L.lo), fabs(L.hi)) <= 0x1p10 &&
         fabs(tt) <= 16.0 && fabs(d) <= 0x1p10 && __builtin_isfinite(qs) && q.RAx > 0.0 && q.twoRAx2 > 0.0;
  c.Z = cover32(Z);
  c.L = cover32(L);
  c.sArc = thin32(q.sArc);
  c.sinA = thin32(q.sinA);
  c.cosA = thin32(q.cosA);
  c.RAx = thin32(q.RAx);
  c.c2 = thin32(q.c2);
  c.s2 = thin32(q.s2);
  c.twoRAx2 = thin32(q.twoRAx2);
  c.RpRAx = thin32(q.RpRAx);
  c.dphi = thin32(q.dphi);
  c.cAx = thin32(q.cAx);
  c.sAx = thin32(q.sAx);
  c.R = thin32(R);
  c.tt = thin32(tt);
  c.t2 = thin32(t2);
  c.d = thin32(d);
  return c;
}

// `neg` selects the drift sign dS = -d.  Outputs as e_enclosure_dom (exact
// FP64 images of the FP32 ends; `out` widened by the point margin).
IA_HD bool e_enclosure32(const EnclIn32& c, bool neg, double sig, Iv* out, Iv* eps_out, Iv* disc_out,
                         Iv* a_out) {
  if (!c.ok) return false;
  const Iv32 DS = neg ? ineg32(c.d) : c.d;
  const Iv32 ZA = iadd32(c.Z, imul32(c.L, c.sArc));
  const Iv32 ZAs = imul32(ZA, c.sinA);
  const Iv32 ZA2 = isqr32(ZA);
  const Iv32 LZA = imul32(c.L, ZA);
  const Iv32 LR = imul32(c.L, c.R);
  const Iv32 L2 = isqr32(c.L);
  const Iv32 PHI1 = ineg32(idiv_pos32(iadd32(ZAs, imul32(imul32(c.L, DS), c.cosA)), c.RAx));
  const Iv32 P2a = imul32(LR, ZA);
  const Iv32 P2b = imul32(imul32(LZA, isub32(c.R, itwice32(DS))), c.c2);
  const Iv32 inner = iadd32(c.RAx, imul32(L2, isub32(c.RpRAx, DS)));
  const Iv32 P2c = imul32(iadd32(ZA2, imul32(DS, inner)), c.s2);
  const Iv32 PHI2 = idiv_pos32(iadd32(isub32(P2a, P2b), P2c), c.twoRAx2);
  const Iv32 EPS = iadd32(imul32(PHI1, c.tt), imul32(PHI2, c.t2));
  *eps_out = {EPS.lo, EPS.hi};
  if (!(fabsf(EPS.lo) <= kSmallTrig32 && fabsf(EPS.hi) <= kSmallTrig32)) return false;
  Iv32 SE, CE;
  sincos_encl_small32(EPS, &SE, &CE);
  const Iv32 SINP = iadd32(imul32(CE, c.sinA), imul32(SE, c.cosA));
  const Iv32 COSP = isub32(imul32(CE, c.cosA), imul32(SE, c.sinA));
  const Iv32 U2 = iadd32(iadd32(iadd32(Iv32{1.0f, 1.0f}, imul32(imul32(itwice32(c.L), SINP), c.tt)), imul32(L2, c.t2)),
                         imul32(isqr32(COSP), c.t2));
  if (!(U2.lo > 0.0f)) return false;
  const Iv32 DELTA = idiv_pos32(DS, isqrt32(U2));
  const Iv32 SPERP = imul32(iadd32(c.dphi, EPS), c.R);
  const Iv32 ZS = isub32(iadd32(c.Z, imul32(c.L, SPERP)), imul32(imul32(DELTA, COSP), c.tt));
  const Iv32 LD = imul32(c.L, DELTA);
  const Iv32 CTAU = isub32(imul32(ZS, c.cAx), imul32(LD, c.sAx));
  const Iv32 Q = iadd32(iadd32(imul32(itwice32(CTAU), c.tt), isqr32(imul32(ZS, c.tt))), isqr32(imul32(LD, c.tt)));
  const Iv32 A = iadd32(c.R, DELTA);
  const Iv32 DISC = isub32(isqr32(A), Q);
  *disc_out = {DISC.lo, DISC.hi};
  *a_out = {A.lo, A.hi};
  if (!(DISC.hi >= 0.0f)) return false;
  const Iv32 DEN = iadd32(A, isqrt32(DISC));
  if (!(DEN.lo > 0.0f)) return false;
  const Iv32 DHAT = isub32(DELTA, idiv_pos32(Q, DEN));
  const Iv E = sig > 0.0 ? Iv{DHAT.lo, DHAT.hi} : Iv{-static_cast<double>(DHAT.hi), -static_cast<double>(DHAT.lo)};
  const double m = 1e-9 * fmax(fabs(E.lo), fabs(E.hi)) + 1e-12;
  *out = {wdn(E.lo - m), wup(E.hi + m)};
  return __builtin_isfinite(out->lo) && __builtin_isfinite(out->hi);
}

// Inclusion: a proof that the per-box test votes for every point value e
// in [E1, E2].  The per-box test (h_contains0, or its FP32 form) votes when
// its interval T = 2E + K E^2, E = [e - b, e + b] rounded outward, has
// T.hi >= 2 G.lo and T.lo <= 2 G.hi.  Outward rounding only widens, so
// T.hi >= 2(e + b) + K.hi s1(e) and T.lo <= 2(e - b) + K.lo s2(e), where s1
// (s2) is the largest square over E when K.hi >= 0 (K.lo < 0) and the
// smallest otherwise.  Both bounds increase with e when
// max|K| (max|e| + b) < 1/2, so checking the first at E1 and the second at
// E2, with outward-rounded arithmetic, covers the whole range.
IA_HD bool votes_everywhere(Iv G, Iv K, double E1, double E2, double b) {
  const double emax = fmax(fabs(E1), fabs(E2));
  if (!(fmax(fabs(K.lo), fabs(K.hi)) * (emax + b) < 0.5)) return false;
  auto sq_big = [&](double e) { return isqr(iadd(ipt(fabs(e)), ipt(b))); };
  auto sq_small = [&](double e) {
    const Iv d = isub(ipt(fabs(e)), ipt(b));
    return isqr(Iv{fmax(d.lo, 0.0), fmax(d.hi, 0.0)});
  };
  const Iv f = iadd(itwice(iadd(ipt(E1), ipt(b))), imul(ipt(K.hi), K.hi >= 0.0 ? sq_big(E1) : sq_small(E1)));
  const Iv g = iadd(itwice(isub(ipt(E2), ipt(b))), imul(ipt(K.lo), K.lo >= 0.0 ? sq_small(E2) : sq_big(E2)));
  return f.lo >= 2.0 * G.lo && g.hi <= 2.0 * G.hi;
}

// Magnitude bound of d^Ax over a triple.  Every term of the point evaluation
// (stereo_vote) is replaced by an upper bound of its absolute value over all
// (z0, tanl) centres of the triple and both drift signs: |z0| <= z, |tanl| <=
// l, |dS| = d, |sinP|, |cosP| <= |sinA| + |cosA| (each is a rotation of
// (sinA, cosA)), u^2 >= 1 - 2 l (|sinA| + |cosA|) tan(tau), A >= R - |delta|,
// and A + sqrt(A^2 - Q) >= alo + sqrt(alo^2 - |Q|) when the root is real
// (a negative discriminant casts no vote).  Only sums, products, quotients
// and roots of non-negative numbers remain, except three subtractions held
// far from cancellation by the checks (u^2 >= 1/4, alo^2 - |Q| >= alo^2 / 4),
// so the bound's own rounding stays below a few hundred ulps, also with the
// divisions by R^Ax and 2 R^Ax^2 taken as products with one rounded
// reciprocal (a few ulps each); the result is
// widened by 2^-29 relative + 1e-12 m, which also covers the point
// evaluation's rounding (the margin of e_enclosure_dom).  Returns false when
// a check fails (no bound).  `eps` bounds |eps|, `disc_lo` bounds the
// discriminant from below and `a_hi` bounds A from above.
struct EMag { double M, eps, disc_lo, a_hi; };

// magnitudes of the pair quantities that e_magnitude uses; sArc and dphi may
// be upper bounds of the absolute values; iRAx is 1 / RAx rounded
struct MagIn { double sa, ca, sArc, dphi, RAx, c2, s2, iRAx, RpRAx, cAx, sAx; };

IA_HD bool e_magnitude_in(const MagIn& q, double R, double tt, double d, Iv Z, Iv L, EMag* out) {
  const double at = fabs(tt), t2 = at * at;
  const double z = fmax(fabs(Z.lo), fabs(Z.hi)), l = fmax(fabs(L.lo), fabs(L.hi));
  const double sa = q.sa, ca = q.ca, S = sa + ca;
  const double za = z + l * q.sArc;
  const double phi1 = (za * sa + (l * d) * ca) * q.iRAx;
  const double phi2 = ((l * R) * za + ((l * za) * (R + 2.0 * d)) * q.c2 +
                       (za * za + d * (q.RAx + (l * l) * (q.RpRAx + d))) * q.s2) * ((0.5 * q.iRAx) * q.iRAx);
  const double eps = phi1 * at + phi2 * t2;
  const double u2 = 1.0 - ((2.0 * l) * S) * at;
  if (!(u2 >= 0.25)) return false;
  const double delta = d / sqrt(u2);
  const double zs = (z + l * (R * (q.dphi + eps))) + (delta * S) * at;
  const double ld = l * delta;
  const double ctau = zs * q.cAx + ld * q.sAx;
  const double Qm = ((2.0 * ctau) * at + (zs * at) * (zs * at)) + (ld * at) * (ld * at);
  const double alo = R - delta;
  if (!(alo > 0.0)) return false;
  const double r = alo * alo - Qm;
  if (!(r >= 0.25 * (alo * alo))) return false;
  const double M = delta + Qm / (alo + sqrt(r));
  out->M = M * (1.0 + 0x1p-29) + 1e-12;
  out->eps = eps * (1.0 + 0x1p-29);
  out->disc_lo = r * (1.0 - 0x1p-29);
  out->a_hi = (R + delta) * (1.0 + 0x1p-29);
  return __builtin_isfinite(out->M) && __builtin_isfinite(out->eps);
}

IA_HD bool e_magnitude(const PairQ& q, double R, double tt, double d, Iv Z, Iv L, EMag* out) {
  const MagIn m = {fabs(q.sinA), fabs(q.cosA), fabs(q.sArc), fabs(q.dphi), q.RAx, fabs(q.c2), fabs(q.s2),
                   1.0 / q.RAx, q.RpRAx, fabs(q.cAx), fabs(q.sAx)};
  return e_magnitude_in(m, R, tt, d, Z, L, out);
}

// The inputs of e_magnitude without the arc angle's atan2: every quantity is
// computed by pair_quantities' operations, except that sinA and cosA are
// products with one rounded reciprocal of RAx (within a few ulps of its
// quotients, far inside e_magnitude's widening), and |dphi| is bounded by
// |y| / x when x > 0 (|atan t| <= |t|; atan2_p is within a few ulps of atan),
// else by pi; |sArc| by R times that.  The widening by 2^-45 covers the few
// ulps.
IA_HD MagIn pair_magnitudes(const Frame& f, const HitRec& h) {
  MagIn m;
  const double py = f.sig * h.py, cps = f.sig * h.cphis, sps = h.sphis;
  const double Dx = h.px - f.xc, Dy = py - f.yc;
  m.RAx = sqrt(Dx * Dx + Dy * Dy);
  const double cAx = Dx * sps - Dy * cps;
  const double sAx = Dx * cps + Dy * sps;
  m.iRAx = 1.0 / m.RAx;
  const double sinA = sAx * m.iRAx, cosA = cAx * m.iRAx;
  const double y = Dx * f.cp0 + Dy * f.sp0, x = Dx * f.sp0 - Dy * f.cp0;
  m.dphi = (x > 0.0 ? fabs(y) / x : kPio2Up * 2.0) * (1.0 + 0x1p-45);
  m.sArc = (f.R * m.dphi) * (1.0 + 0x1p-45);
  m.sa = fabs(sinA);
  m.ca = fabs(cosA);
  m.c2 = fabs(cosA * cosA - sinA * sinA);
  m.s2 = fabs(2.0 * sinA * cosA);
  m.RpRAx = f.R + m.RAx;
  m.cAx = fabs(cAx);
  m.sAx = fabs(sAx);
  return m;
}

// H test of reading 8 over E = [-M, M] widened by the band: false when the
// pair can vote in no box whose |e| is at most M
IA_HD bool h_may_vote_mag(Iv G, Iv K, double M, double band) {
  const double b = wup(M + band);
  const Iv Eb = {-b, b};
  const Iv Hb = isub(itwice(G), iadd(itwice(Eb), imul(K, isqr(Eb))));
  return Hb.lo <= 0.0 && 0.0 <= Hb.hi;
}

// Class of a (triple, stereo hit) pair at an FP64 level: 0 when no box of
// the triple can get the hit's vote, 1 when every box gets it, 2 when the
// boxes must be evaluated one by one.  Class 1 needs, for one drift sign,
// a well-conditioned point evaluation everywhere on the rectangle (the
// discriminant of d^Ax above A^2 / 4) and the inclusion proof above over
// the enclosure of e.
// The class is decided in two stages: stereo_quick_class (the magnitude
// bound of e, which excludes most pairs that can be excluded at a small part
// of an enclosure's cost; 0 or -1 for undecided) and stereo_pass_class (the
// FP32 enclosure, e_enclosure32, per drift sign).  With `cnt` set, cnt[0] counts the enclosure
// passes and cnt[1] the inclusion proofs evaluated.
IA_HD int stereo_quick_class_in(const MagIn& m, Iv G, const Frame& f, const HitRec& h, Iv Z, Iv L) {
  EMag em;
  if (e_magnitude_in(m, f.R, h.tant, h.d, Z, L, &em) && !h_may_vote_mag(G, f.K, em.M, h.band)) return 0;
  return -1;
}

IA_HD int stereo_quick_class(const PairQ& q, const Frame& f, const HitRec& h, Iv Z, Iv L) {
  EMag em;
  if (e_magnitude(q, f.R, h.tant, h.d, Z, L, &em) && !h_may_vote_mag(Iv{q.Glo, q.Ghi}, f.K, em.M, h.band))
    return 0;
  return -1;
}

// `signs` (bit 0: dS = +d, bit 1: dS = -d): the drift signs left open; a
// sign outside it casts no vote in any box of the triple and is skipped.
// Exclusions and inclusions from an enclosure of d^Ax are taken only where
// the discriminant of Eq. defdiAX_b stays above A^2 / 4 over it: there the
// square root and the quotient Q / (A + sqrt(disc)) are well conditioned, so
// the point evaluation's rounding stays far inside the 1e-9 |e| + 1e-12 m
// margin (checked against long-double evaluations); elsewhere the boxes are
// evaluated one by one.
IA_HD bool well_conditioned(Iv DISC, Iv A) { return A.lo > 0.0 && DISC.lo > 0.25 * A.lo * A.lo; }

IA_HD int stereo_pass_class(const PairQ& q, const Frame& f, const HitRec& h, Iv Z, Iv L, int signs = 3,
                            int32_t* cnt = nullptr) {
  const Iv G = {q.Glo, q.Ghi};
  const double tt = h.tant, t2 = tt * tt;
  const EnclIn32 c = encl_in32(q, f.R, tt, t2, h.d, Z, L);
  bool may = false;
  // passes 0 and 1: each drift sign.  One loop body, kept rolled, holds the
  // enclosure's registers once.
#pragma unroll 1
  for (int si = 0; si < 2; ++si) {
    if (!((signs >> si) & 1)) continue;
    Iv E, EPS, DISC, A;
    const bool ok = e_enclosure32(c, si != 0, f.sig, &E, &EPS, &DISC, &A);
    if (cnt) ++cnt[0];
    const bool try_incl = ok && well_conditioned(DISC, A);
    if (cnt && try_incl) ++cnt[1];
    if (try_incl && votes_everywhere(G, f.K, E.lo, E.hi, h.band)) return 1;
    bool in = true;                      // the test cannot be excluded on this pass
    if (try_incl) {
      const Iv Eb = {wdn(E.lo - h.band), wup(E.hi + h.band)};
      const Iv Hb = isub(itwice(G), iadd(itwice(Eb), imul(f.K, isqr(Eb))));
      in = Hb.lo <= 0.0 && 0.0 <= Hb.hi;
    }
    may = may || in;
  }
  return may ? 2 : 0;
}

IA_HD int triple_vote_class(const PairQ& q, const Frame& f, const HitRec& h, Iv Z, Iv L, int32_t* cnt = nullptr) {
  const int c = stereo_quick_class(q, f, h, Z, L);
  return c >= 0 ? c : stereo_pass_class(q, f, h, Z, L, 3, cnt);
}

// false only when no box of the triple can get this stereo hit's vote
IA_HD bool triple_may_vote(const PairQ& q, const Frame& f, const HitRec& h, Iv Z, Iv L) {
  return triple_vote_class(q, f, h, Z, L) != 0;
}

// ---------------------------------------------------------------------------
// FP32 levels.  A stereo pair's (triple, hit) quantities are the FP64 ones
// above, rounded to FP32 (G outward, points to nearest); the (z0, tanl) part
// of d^Ax runs in FP32 in the operation order of stereo_vote, and the vote
// test is the FP32 interval test with the band widened by a slack that
// bounds |e32 - e64|.  The FP32 evaluation is used only where that bound
// holds (R <= kR32Max, |eps| <= 1, positive discriminant, finite result);
// elsewhere the pair votes.  FP32 votes thus contain the FP64 votes.
constexpr double kR32Max = 2048.0;

struct PairQ32 {
  float Glo, Ghi, sArc, dphi, RAx, sinA, cosA, sAx, cAx, c2, s2, twoRAx2, RpRAx, tt, d, bs;
};

IA_HD PairQ32 pair_q32(const PairQ& q, const HitRec& h, float slack32) {
  PairQ32 r;
  r.Glo = rd32(q.Glo); r.Ghi = ru32(q.Ghi);
  r.sArc = static_cast<float>(q.sArc); r.dphi = static_cast<float>(q.dphi);
  r.RAx = static_cast<float>(q.RAx); r.sinA = static_cast<float>(q.sinA);
  r.cosA = static_cast<float>(q.cosA); r.sAx = static_cast<float>(q.sAx);
  r.cAx = static_cast<float>(q.cAx); r.c2 = static_cast<float>(q.c2); r.s2 = static_cast<float>(q.s2);
  r.twoRAx2 = static_cast<float>(q.twoRAx2); r.RpRAx = static_cast<float>(q.RpRAx);
  r.tt = static_cast<float>(h.tant);
  r.d = static_cast<float>(h.d);
  r.bs = wup32(ru32(h.band) + slack32);
  return r;
}

// FP32 levels evaluate the whole predicate in FP32: the box's (d0, phi0,
// kappa) ranges rounded outward, its centre rounded to nearest, G of Eq.
// ApoVote in FP32 intervals with the FP32 sine enclosure, the transverse
// quantities of d^Ax in FP32 (sinf32, cosf32, atan2f32), and the band
// widened by slack + 2^-24 R, a bound on |e32 - e64| (the transverse
// quantities are of size R with FP32 rounding).  No class proofs run at
// such levels; the per-box test is stereo_vote32 on these quantities.
struct Frame32 {
  Iv32 K, Dd, Fi;
  float sig, R, xc, yc, sp0, cp0;
};

IA_HD Frame32 frame32_of(const Frame& f) {
  Frame32 g;
  g.Dd = {rd32(f.Dd.lo), ru32(f.Dd.hi)};
  g.Fi = {rd32(f.Fi.lo), ru32(f.Fi.hi)};
  g.K = {rd32(f.K.lo), ru32(f.K.hi)};
  const float c0 = static_cast<float>(0.5 * (f.Dd.lo + f.Dd.hi)), c1 = static_cast<float>(0.5 * (f.Fi.lo + f.Fi.hi));
  float kap = static_cast<float>(0.5 * (f.K.lo + f.K.hi)), sig = 1.0f;
  if (kap < 0.0f) sig = -1.0f;
  if (kap == 0.0f) { kap = 0x1p-30f; sig = 1.0f; }
  const float kp = sig * kap, d0p = sig * c0;
  g.sp0 = sig * sinf32(c1);
  g.cp0 = cosf32(c1);
  g.R = 1.0f / kp;
  const float Rd = g.R + d0p;
  g.xc = -(Rd * g.sp0);
  g.yc = Rd * g.cp0;
  g.sig = sig;
  return g;
}

IA_HD Iv32 residual_G32(const Frame32& f, const HitRec& h) {
  const Iv32 P = {rd32(h.phip), ru32(h.phip)};
  const Iv32 Ar = {wdn32(f.Fi.lo - P.hi), wup32(f.Fi.hi - P.lo)};
  const Iv32 S = sin_encl32(Ar.lo, Ar.hi);
  const Iv32 r = {rd32(h.r), ru32(h.r)};
  const Iv32 rS = imul32(S, r);
  const Iv32 D2 = isqr32(f.Dd);
  const Iv32 T0 = iadd32(D2, Iv32{rd32(h.r2lo), ru32(h.r2hi)});
  const Iv32 T = {0.5f * T0.lo, 0.5f * T0.hi};
  const Iv32 KT = imul32(f.K, T);
  const Iv32 KD1 = iadd32(imul32(f.K, f.Dd), Iv32{1.0f, 1.0f});
  return iadd32(iadd32(KT, imul32(KD1, rS)), f.Dd);
}

// an axial pair at an FP32 level: e = +-d exactly, no slack
IA_HD int axial_class32(const Frame32& f, const HitRec& h) {
  const Iv32 G = residual_G32(f, h);
  const float b = ru32(h.band);
  for (int si = 0; si < 2; ++si) {
    const double e = static_cast<double>(f.sig) * (si == 0 ? h.d : -h.d);
    const Iv32 E = {wdn32(rd32(e) - b), wup32(ru32(e) + b)};
    const Iv32 H = isub32(itwice32(G), iadd32(itwice32(E), imul32(f.K, isqr32(E))));
    if (H.lo <= 0.0f && 0.0f <= H.hi) return 1;
  }
  return 0;
}

// the staged record of a stereo pair at an FP32 level
IA_HD PairQ32 pair_q32_f32(const Frame32& f, const HitRec& h, float slack32) {
  PairQ32 r;
  const Iv32 G = residual_G32(f, h);
  const float py = f.sig * static_cast<float>(h.py), cps = f.sig * static_cast<float>(h.cphis);
  const float sps = static_cast<float>(h.sphis);
  const float Dx = static_cast<float>(h.px) - f.xc, Dy = py - f.yc;
  const float RAx = sqrtf(Dx * Dx + Dy * Dy);
  const float cAx = Dx * sps - Dy * cps;
  const float sAx = Dx * cps + Dy * sps;
  const float sinA = sAx / RAx, cosA = cAx / RAx;
  const float dphi = atan2f32(Dx * f.cp0 + Dy * f.sp0, Dx * f.sp0 - Dy * f.cp0);
  r.Glo = G.lo;
  r.Ghi = G.hi;
  r.sArc = f.R * dphi;
  r.dphi = dphi;
  r.RAx = RAx;
  r.sinA = sinA;
  r.cosA = cosA;
  r.sAx = sAx;
  r.cAx = cAx;
  r.c2 = cosA * cosA - sinA * sinA;
  r.s2 = 2.0f * sinA * cosA;
  r.twoRAx2 = 2.0f * (RAx * RAx);
  r.RpRAx = f.R + RAx;
  r.tt = static_cast<float>(h.tant);
  r.d = static_cast<float>(h.d);
  r.bs = wup32(wup32(ru32(h.band) + slack32) + f.R * 0x1p-24f);
  return r;
}

// a staged (triple, stereo hit) record at FP64 levels: the pair quantities
// and the hit's tan(tau), drift and band (128 bytes)
struct RecD {
  double q[13];
  double tt, d, band;
};
// per-triple frame values the per-box evaluation needs: R, sign, kappa interval
struct TriFrame { double R, sig, Klo, Khi; };

IA_HD bool stereo_vote32(const PairQ32& q, float R, float sig, Iv32 K, float z0, float lam, float lamR,
                         float lam2) {
  const float tt = q.tt, t2 = tt * tt;
  const float zA = z0 + lam * q.sArc;
  const float zAs = zA * q.sinA;
  const float zA2 = zA * zA;
  const float lzA = lam * zA;
  const Iv32 G = {q.Glo, q.Ghi};
  bool vote = false;
#pragma unroll
  for (int si = 0; si < 2; ++si) {
    const float dS = si == 0 ? q.d : -q.d;
    const float Phi1 = -(zAs + (lam * dS) * q.cosA) / q.RAx;
    const float Phi2n = lamR * zA - (lzA * (R - 2.0f * dS)) * q.c2 + (zA2 + dS * (q.RAx + lam2 * (q.RpRAx - dS))) * q.s2;
    const float Phi2 = Phi2n / q.twoRAx2;
    const float eps = Phi1 * tt + Phi2 * t2;
    if (!(fabsf(eps) <= 1.0f)) { vote = true; continue; }
    const float se = sin1_32(eps), ce = cos1_32(eps);
    const float sinP = q.sinA * ce + q.cosA * se, cosP = q.cosA * ce - q.sinA * se;
    const float u = sqrtf(((1.0f + ((2.0f * lam) * sinP) * tt) + lam2 * t2) + (cosP * cosP) * t2);
    const float delta = dS / u;
    const float sperp = R * (q.dphi + eps);
    const float zS = (z0 + lam * sperp) - (delta * cosP) * tt;
    const float ld = lam * delta;
    const float ctau = zS * q.cAx - ld * q.sAx;
    const float a1 = zS * tt, a2 = ld * tt;
    const float Q = ((2.0f * ctau) * tt + a1 * a1) + a2 * a2;
    const float A = R + delta;
    const float disc = A * A - Q;
    if (!(disc > 0.0f)) { vote = true; continue; }
    const float e = sig * (delta - Q / (A + sqrtf(disc)));
    if (!__builtin_isfinite(e)) { vote = true; continue; }
    const Iv32 E = {wdn32(e - q.bs), wup32(e + q.bs)};
    const Iv32 Hv = isub32(itwice32(G), iadd32(itwice32(E), imul32(K, isqr32(E))));
    if (Hv.lo <= 0.0f && 0.0f <= Hv.hi) vote = true;
  }
  return vote;
}

// Class (0, 1, 2 as in triple_vote_class) of a (triple, stereo hit) pair at
// an FP32 level.  Exclusion: the enclosure of e over the centre rectangle
// must show that every box stays in the FP32 domain (|eps| <= 0.99, a
// discriminant above 1e-3 A^2, far beyond FP32 rounding); its FP32 image is
// widened by band + 2 slack (one slack for |e32 - e64|, one to spare for
// FP32 rounding) before the FP32 interval test.  Inclusion: the proof of
// votes_everywhere holds for FP32 outward rounding as well; it is applied to
// the FP32 G, K and band (exact in FP64) over [E1 - slack, E2 + slack],
// which holds every box's e32 (a box outside the FP32 domain votes anyway).
// Two stages as at FP64 levels; the quick stage also gives class 1 to a
// triple outside the FP32 domain, and its exclusion needs every box inside
// the domain.
IA_HD int stereo_quick_class32_in(const MagIn& m, Iv G64, const Frame& f, const HitRec& h, Iv Z, Iv L,
                                   float slack32) {
  if (!(f.R <= kR32Max)) return 1;
  EMag em;
  if (e_magnitude_in(m, f.R, h.tant, h.d, Z, L, &em) && em.eps <= 0.99 && em.disc_lo > 1e-3 * em.a_hi * em.a_hi) {
    const Iv32 G = to32(G64);
    const Iv32 K = to32(f.K);
    const float bs2 = wup32(ru32(h.band) + 2.0f * slack32);
    const float m32 = ru32(em.M);
    const Iv32 Eb = {wdn32(-m32 - bs2), wup32(m32 + bs2)};
    const Iv32 Hb = isub32(itwice32(G), iadd32(itwice32(Eb), imul32(K, isqr32(Eb))));
    if (!(Hb.lo <= 0.0f && 0.0f <= Hb.hi)) return 0;
  }
  return -1;
}

IA_HD int stereo_quick_class32(const PairQ& q, const Frame& f, const HitRec& h, Iv Z, Iv L, float slack32) {
  if (!(f.R <= kR32Max)) return 1;
  EMag em;
  if (e_magnitude(q, f.R, h.tant, h.d, Z, L, &em) && em.eps <= 0.99 && em.disc_lo > 1e-3 * em.a_hi * em.a_hi) {
    const Iv32 G = to32(Iv{q.Glo, q.Ghi});
    const Iv32 K = to32(f.K);
    const float bs2 = wup32(ru32(h.band) + 2.0f * slack32);
    const float m32 = ru32(em.M);
    const Iv32 Eb = {wdn32(-m32 - bs2), wup32(m32 + bs2)};
    const Iv32 Hb = isub32(itwice32(G), iadd32(itwice32(Eb), imul32(K, isqr32(Eb))));
    if (!(Hb.lo <= 0.0f && 0.0f <= Hb.hi)) return 0;
  }
  return -1;
}

IA_HD int stereo_pass_class32(const PairQ& q, const Frame& f, const HitRec& h, Iv Z, Iv L, float slack32,
                              int signs = 3, int32_t* cnt = nullptr) {
  const Iv32 G = to32(Iv{q.Glo, q.Ghi});
  const Iv32 K = to32(f.K);
  const float bs = wup32(ru32(h.band) + slack32);
  const float bs2 = wup32(ru32(h.band) + 2.0f * slack32);
  const double tt = h.tant, t2 = tt * tt;
  const EnclIn32 c = encl_in32(q, f.R, tt, t2, h.d, Z, L);
  bool may = false;
  // passes 0 and 1: each drift sign (one rolled loop body, as in
  // stereo_pass_class)
#pragma unroll 1
  for (int si = 0; si < 2; ++si) {
    if (!((signs >> si) & 1)) continue;
    Iv E, EPS, DISC, A;
    const bool ok = e_enclosure32(c, si != 0, f.sig, &E, &EPS, &DISC, &A);
    if (cnt) ++cnt[0];
    const bool try_incl = ok && well_conditioned(DISC, A);
    if (cnt && try_incl) ++cnt[1];
    if (try_incl && votes_everywhere(Iv{G.lo, G.hi}, Iv{K.lo, K.hi}, wdn(E.lo - slack32), wup(E.hi + slack32), bs))
      return 1;
    // excluded only when every box stays in the FP32 domain and the widened
    // FP32 test fails over the whole enclosure
    bool in = true;
    if (try_incl && fabs(EPS.lo) <= 0.99 && fabs(EPS.hi) <= 0.99 && DISC.lo > 1e-3 * A.hi * A.hi) {
      const Iv32 Eb = {wdn32(rd32(E.lo) - bs2), wup32(ru32(E.hi) + bs2)};
      const Iv32 Hb = isub32(itwice32(G), iadd32(itwice32(Eb), imul32(K, isqr32(Eb))));
      in = Hb.lo <= 0.0f && 0.0f <= Hb.hi;
    }
    may = may || in;
  }
  return may ? 2 : 0;
}

IA_HD int triple_vote_class32(const PairQ& q, const Frame& f, const HitRec& h, Iv Z, Iv L, float slack32,
                              int32_t* cnt = nullptr) {
  const int c = stereo_quick_class32(q, f, h, Z, L, slack32);
  return c >= 0 ? c : stereo_pass_class32(q, f, h, Z, L, slack32, 3, cnt);
}

// What the parent-level enclosures of d^Ax give the first stage of the child
// triples' classification (parent_range_signs), per drift sign s: when
// ok[s] is set, [wlo[s], whi[s]] holds the per-box H test's term
// 2 E + kappa E^2 for every child box centre (E the point value of d^Ax
// widened by the band, kappa over the parent); ok[s] is 0 where no range is
// available (axial hits, FP32 levels, failed enclosures).
struct ParentE {
  double wlo[2], whi[2];
  int32_t ok[2];
};

// First-stage exclusion of a stereo pair at an FP64 refinement level with
// the parent's ranges (ParentE), which hold the triple's boxes (its box
// centres are among the parent's child centres): the set of drift signs for
// which the per-box H test may pass for a term in [wlo, whi] with the outer
// G (none: class 0; one: the second stage runs that sign's pass only).  The
// per-box test computes wdn(2 G.lo - X.hi) and wup(2 G.hi - X.lo) for its
// term X, which lies inside [wlo, whi] (the same outward-rounded operations
// on narrower intervals), with G inside the outer G; both roundings are
// monotone, so the bounds below carry over to every box.
IA_HD int parent_range_signs(const ParentE& pe, Iv Go) {
  int open = 0;
  for (int si = 0; si < 2; ++si)
    if (!pe.ok[si] || !(wdn(2.0 * Go.lo - pe.whi[si]) > 0.0 || wup(2.0 * Go.hi - pe.wlo[si]) < 0.0))
      open |= 1 << si;
  return open;
}

// The two stages of a (triple, hit) pair's class as the kernels run them.
// Stage 1 (k_classify): the outer G (residual_G_outer); an axial pair is
// decided exactly, with the exact G only when the outer one does not already
// exclude both signs; a stereo pair is excluded by parent_range_signs (FP64
// refinement levels, with the parent's ranges `pe`) or by the magnitude
// bound from pair_magnitudes and the outer G, else deferred: the result is
// then minus the set of drift signs left open (-3 both, -1 +d, -2 -d).
// Outside the FP32 domain a stereo pair votes (1); without the proofs
// (`filter` 0) it is class 2.  cnt[kCwG ..] counts the work when set.
template <bool F32>
IA_HD int pair_stage1(const Frame& f, const GTri& g, const HitRec& h, Iv Z, Iv L, int32_t filter, float slack32,
                      int32_t* cnt, const ParentE* pe = nullptr) {
  if constexpr (F32) {
    // FP32 levels: no class proofs; an axial pair's class is exact, a
    // stereo pair outside the FP32 domain votes in every box
    const Frame32 g32 = frame32_of(f);
    if (cnt) ++cnt[kCwG];
    if (h.axial) return axial_class32(g32, h);
    return g32.R <= static_cast<float>(kR32Max) ? 2 : 1;
  }
  const Iv Go = residual_G_outer(f, g, h);
  if (cnt) ++cnt[kCwG];
  if (h.axial) {
    if (cnt) ++cnt[kCwAxial];
    if (!h_contains0(Go, f.K, f.sig * h.d, h.band) && !h_contains0(Go, f.K, f.sig * (-h.d), h.band)) return 0;
    if (cnt) ++cnt[kCwGExact];
    const Iv G = residual_G(f, h);
    return (h_contains0(G, f.K, f.sig * h.d, h.band) || h_contains0(G, f.K, f.sig * (-h.d), h.band)) ? 1 : 0;
  }
  if (F32 && !(f.R <= kR32Max)) return 1;
  if (!filter) return 2;
  const int signs = (!F32 && pe) ? parent_range_signs(*pe, Go) : 3;
  if (!signs) return 0;
  if (cnt) { ++cnt[kCwPairQ]; ++cnt[kCwMag]; }
  const MagIn m = pair_magnitudes(f, h);
  const int c = F32 ? stereo_quick_class32_in(m, Go, f, h, Z, L, slack32) : stereo_quick_class_in(m, Go, f, h, Z, L);
  return c >= 0 ? c : -signs;
}

// Stage 2 (k_classify_defer): the exact G and pair quantities, then the
// enclosure passes of the drift signs stage 1 left open.  cnt[0] counts
// enclosures, cnt[1] inclusion proofs.
template <bool F32>
IA_HD int pair_stage2(const Frame& f, const HitRec& h, Iv Z, Iv L, float slack32, int signs, int32_t* cnt) {
  const PairQ q = pair_quantities(f, h, residual_G(f, h));
  return F32 ? stereo_pass_class32(q, f, h, Z, L, slack32, signs, cnt)
             : stereo_pass_class(q, f, h, Z, L, signs, cnt);
}

// (z0, tanl) centre ranges of the boxes of one parent
IA_HD void centre_ranges(const BoxD& P, const uint32_t m[5], Iv* Z, Iv* L) {
  double lo, hi, lo2, hi2;
  child_edge(P.lo[3], P.hi[3], m[3], 0, &lo, &hi);
  child_edge(P.lo[3], P.hi[3], m[3], m[3] - 1, &lo2, &hi2);
  *Z = {0.5 * (lo + hi), 0.5 * (lo2 + hi2)};
  child_edge(P.lo[4], P.hi[4], m[4], 0, &lo, &hi);
  child_edge(P.lo[4], P.hi[4], m[4], m[4] - 1, &lo2, &hi2);
  *L = {0.5 * (lo + hi), 0.5 * (lo2 + hi2)};
}

// ---------------------------------------------------------------------------
// Parent-level exclusion (refinement levels): can a hit vote for any box of
// a parent at all?  Every point operation of triple_frame and
// pair_quantities is mirrored by the same interval operation over the
// parent's child-triple centres (whose end points are the first and last
// child centre of each dimension, exactly as the children compute them).
// Round-to-nearest is monotone and every interval end point is rounded
// outward by at least one ulp, so each interval contains the floating-point
// value every child triple computes; the sin and cos enclosures carry their
// margin, and atan2 is enclosed by its values at the corners of its argument
// box plus 1e-13 (the whole [-pi, pi] when that box meets the negative x axis).
struct FrameIv {
  Iv K, Dd, Fi;                 // the parent's kappa, d0, phi0 ranges (for G)
  double sig;
  Iv R, XC, YC, SP0, CP0;
};
struct PairQIv { Iv sArc, dphi, RAx, sinA, cosA, sAx, cAx, c2, s2, twoRAx2, RpRAx; };

IA_HD Iv atan2_encl(Iv Y, Iv X) {
  if (X.lo <= 0.0 && Y.lo <= 0.0 && Y.hi >= 0.0) return {-kPio2Up * 2.0, kPio2Up * 2.0};
  const double a = atan2_p(Y.lo, X.lo), b = atan2_p(Y.lo, X.hi), c = atan2_p(Y.hi, X.lo), d = atan2_p(Y.hi, X.hi);
  return {fmin(fmin(a, b), fmin(c, d)) - 1e-13, fmax(fmax(a, b), fmax(c, d)) + 1e-13};
}

// false when the children's kappa centres are not all of one sign (no frame)
IA_HD bool parent_frame(const BoxD& P, const uint32_t m[5], FrameIv* f) {
  double c[3][2];
  for (int j = 0; j < 3; ++j) {
    double lo, hi, lo2, hi2;
    child_edge(P.lo[j], P.hi[j], m[j], 0, &lo, &hi);
    child_edge(P.lo[j], P.hi[j], m[j], m[j] - 1, &lo2, &hi2);
    c[j][0] = 0.5 * (lo + hi);
    c[j][1] = 0.5 * (lo2 + hi2);
  }
  f->Dd = {P.lo[0], P.hi[0]};
  f->Fi = {P.lo[1], P.hi[1]};
  f->K = {P.lo[2], P.hi[2]};
  double sig;
  if (c[2][0] > 0.0) sig = 1.0;
  else if (c[2][1] < 0.0) sig = -1.0;
  else return false;
  const Iv KP = sig > 0.0 ? Iv{c[2][0], c[2][1]} : Iv{-c[2][1], -c[2][0]};
  const Iv D0P = sig > 0.0 ? Iv{c[0][0], c[0][1]} : Iv{-c[0][1], -c[0][0]};
  const Iv R = {wdn(1.0 / KP.hi), wup(1.0 / KP.lo)};
  const Iv S1 = sin_encl(c[1][0], c[1][1]), C1 = cos_encl(c[1][0], c[1][1]);
  f->SP0 = sig > 0.0 ? S1 : ineg(S1);
  f->CP0 = C1;
  const Iv RD = iadd(R, D0P);
  f->XC = ineg(imul(RD, f->SP0));
  f->YC = imul(RD, f->CP0);
  f->R = R;
  f->sig = sig;
  return true;
}

IA_HD bool parent_pairq(const FrameIv& f, const HitRec& h, PairQIv* q) {
  const double py = f.sig * h.py, cps = f.sig * h.cphis, sps = h.sphis;
  const Iv Dx = isub(ipt(h.px), f.XC), Dy = isub(ipt(py), f.YC);
  q->RAx = isqrt(iadd(isqr(Dx), isqr(Dy)));
  if (!(q->RAx.lo > 0.0)) return false;
  q->cAx = isub(imul_pt(Dx, sps), imul_pt(Dy, cps));
  q->sAx = iadd(imul_pt(Dx, cps), imul_pt(Dy, sps));
  q->sinA = idiv_pos2(q->sAx, q->RAx);
  q->cosA = idiv_pos2(q->cAx, q->RAx);
  q->dphi = atan2_encl(iadd(imul(Dx, f.CP0), imul(Dy, f.SP0)), isub(imul(Dx, f.SP0), imul(Dy, f.CP0)));
  q->sArc = imul(f.R, q->dphi);
  q->c2 = isub(isqr(q->cosA), isqr(q->sinA));
  q->s2 = itwice(imul(q->sinA, q->cosA));
  q->twoRAx2 = itwice(isqr(q->RAx));
  q->RpRAx = iadd(f.R, q->RAx);
  return true;
}

// e_enclosure_dom with interval pair quantities and radius
IA_HD bool e_enclosure_iq(const PairQIv& q, Iv R, double sig, double tt, double t2, Iv DS, Iv Z, Iv L, Iv* out,
                          Iv* eps_out, Iv* disc_out, Iv* a_out) {
  const Iv ZA = iadd(Z, imul(L, q.sArc));
  const Iv ZAs = imul(ZA, q.sinA);
  const Iv ZA2 = isqr(ZA);
  const Iv LZA = imul(L, ZA);
  const Iv LR = imul(L, R);
  const Iv L2 = isqr(L);
  const Iv PHI1 = ineg(idiv_pos2(iadd(ZAs, imul(imul(L, DS), q.cosA)), q.RAx));
  const Iv P2a = imul(LR, ZA);
  const Iv P2b = imul(imul(LZA, isub(R, itwice(DS))), q.c2);
  const Iv inner = iadd(q.RAx, imul(L2, isub(q.RpRAx, DS)));
  const Iv P2c = imul(iadd(ZA2, imul(DS, inner)), q.s2);
  const Iv PHI2 = idiv_pos2(iadd(isub(P2a, P2b), P2c), q.twoRAx2);
  const Iv EPS = iadd(imul_pt(PHI1, tt), imul_pt(PHI2, t2));
  *eps_out = EPS;
  if (!(fabs(EPS.lo) < 1e5 && fabs(EPS.hi) < 1e5)) return false;
  Iv SE, CE;
  if (fabs(EPS.lo) <= kSmallTrig && fabs(EPS.hi) <= kSmallTrig) {
    sincos_encl_small(EPS, &SE, &CE);
  } else {
    SE = sin_encl(EPS.lo, EPS.hi);
    CE = cos_encl(EPS.lo, EPS.hi);
  }
  const Iv SINP = iadd(imul(CE, q.sinA), imul(SE, q.cosA));
  const Iv COSP = isub(imul(CE, q.cosA), imul(SE, q.sinA));
  const Iv U2 = iadd(iadd(iadd(ipt(1.0), imul_pt(imul(itwice(L), SINP), tt)), imul_pt(L2, t2)),
                     imul_pt(isqr(COSP), t2));
  if (!(U2.lo > 0.0)) return false;
  const Iv DELTA = idiv_pos2(DS, isqrt(U2));
  const Iv SPERP = imul(iadd(q.dphi, EPS), R);
  const Iv ZS = isub(iadd(Z, imul(L, SPERP)), imul_pt(imul(DELTA, COSP), tt));
  const Iv LD = imul(L, DELTA);
  const Iv CTAU = isub(imul(ZS, q.cAx), imul(LD, q.sAx));
  const Iv Q = iadd(iadd(imul_pt(itwice(CTAU), tt), isqr(imul_pt(ZS, tt))), isqr(imul_pt(LD, tt)));
  const Iv A = iadd(R, DELTA);
  const Iv DISC = isub(isqr(A), Q);
  *disc_out = DISC;
  *a_out = A;
  if (!(DISC.hi >= 0.0)) return false;
  const Iv DEN = iadd(A, isqrt(DISC));
  if (!(DEN.lo > 0.0)) return false;
  const Iv DHAT = isub(DELTA, idiv_pos2(Q, DEN));
  const Iv E = sig > 0.0 ? DHAT : ineg(DHAT);
  const double mg = 1e-9 * fmax(fabs(E.lo), fabs(E.hi)) + 1e-12;
  *out = {wdn(E.lo - mg), wup(E.hi + mg)};
  return __builtin_isfinite(out->lo) && __builtin_isfinite(out->hi);
}

// false only when the hit can vote for no box of the parent's children
// (at FP32 levels, under the FP32 definition: out-of-domain boxes vote).
// At FP64 levels the two drift signs get one enclosure each (inside the
// combined one, so at least as sharp), written to `pe` when set.
template <bool F32>
IA_HD bool parent_may_vote(const BoxD& P, const uint32_t m[5], const HitRec& h, float slack32,
                           ParentE* pe = nullptr) {
  if (pe) pe->ok[0] = pe->ok[1] = 0;
  if (!votes_now(h)) return false;
  FrameIv f;
  if (!parent_frame(P, m, &f)) return true;
  Frame fg;                                     // the parent box's ranges for G
  fg.K = f.K;
  fg.Dd = f.Dd;
  fg.Fi = f.Fi;
  const Iv G = residual_G(fg, h);
  if (h.axial)
    return h_contains0(G, f.K, f.sig * h.d, h.band) || h_contains0(G, f.K, f.sig * (-h.d), h.band);
  if (F32 && !(f.R.hi <= kR32Max)) return true;
  PairQIv q;
  if (!parent_pairq(f, h, &q)) return true;
  Iv Z, L;
  centre_ranges(P, m, &Z, &L);
  const double tt = h.tant, t2 = tt * tt;
  Iv E, EPS, DISC, A;
  if constexpr (!F32) {
    bool may = false;
    for (int si = 0; si < 2; ++si) {
      const double ds = si == 0 ? h.d : -h.d;
      const bool ok = e_enclosure_iq(q, f.R, f.sig, tt, t2, Iv{ds, ds}, Z, L, &E, &EPS, &DISC, &A);
      bool in = true;
      if (ok && well_conditioned(DISC, A)) {
        const Iv Eb = {wdn(E.lo - h.band), wup(E.hi + h.band)};
        const Iv X = iadd(itwice(Eb), imul(f.K, isqr(Eb)));
        const Iv Hb = isub(itwice(G), X);
        in = Hb.lo <= 0.0 && 0.0 <= Hb.hi;
        if (pe) {
          pe->wlo[si] = X.lo;
          pe->whi[si] = X.hi;
          pe->ok[si] = 1;
        }
      }
      may = may || in;
    }
    return may;
  }
  if (!e_enclosure_iq(q, f.R, f.sig, tt, t2, Iv{-h.d, h.d}, Z, L, &E, &EPS, &DISC, &A)) return true;
  if constexpr (F32) {
    if (!(fabs(EPS.lo) <= 0.99 && fabs(EPS.hi) <= 0.99 && DISC.lo > 1e-3 * A.hi * A.hi && well_conditioned(DISC, A)))
      return true;
    const Iv32 G32 = to32(G), K32 = to32(f.K);
    const float bs2 = wup32(ru32(h.band) + 2.0f * slack32);
    const Iv32 Eb = {wdn32(rd32(E.lo) - bs2), wup32(ru32(E.hi) + bs2)};
    const Iv32 Hb = isub32(itwice32(G32), iadd32(itwice32(Eb), imul32(K32, isqr32(Eb))));
    return Hb.lo <= 0.0f && 0.0f <= Hb.hi;
  }
  return true;
}

// ---------------------------------------------------------------------------
// hit preparation.  One thread per hit; also clears the vote and lower-bound
// histograms and the per-triple bounds.  With `ev` set it starts an event:
// resets the event state, writes the search range box and marks every hit
// unassigned.
__global__ void k_prep(const double* __restrict__ hits, const uint8_t* __restrict__ active, EvView vw,
                       HitRec* __restrict__ out, uint32_t* __restrict__ hist, uint32_t* __restrict__ lbh,
                       int32_t* __restrict__ tlb, int32_t* __restrict__ tn2, uint32_t* __restrict__ status,
                       int64_t* __restrict__ n_bad, EventState* __restrict__ ev, int32_t* __restrict__ n_out,
                       BoxD* __restrict__ range_dst, BoxD range, int32_t* __restrict__ assigned,
                       double xr, double yr, const int32_t* __restrict__ rows) {
  // rows (resident pools): the events to prepare, one per grid row
  const int e = rows ? rows[blockIdx.y] : static_cast<int>(blockIdx.y);
  const int32_t beg = vw.beg(e), n_hits = vw.count(e), n_bins = n_hits + 1;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t stride = gridDim.x * blockDim.x;
  // offsets are checked against the sizes the strides were laid out for; an
  // event outside them is stopped (no kernel touches it) and flagged
  const bool bad_ev = vw.max_hits > 0 && (n_hits < 0 || n_hits > vw.max_hits || beg < 0 ||
                                          static_cast<int64_t>(beg) + n_hits > vw.n_total);
  if (ev && i == 0) {
    EventState es{};
    es.t_cut = INT32_MAX;
    if (bad_ev) {
      es.done = 1;
      atomicOr(status, kStBadOffsets);
    }
    ev[e] = es;
    if (n_out) n_out[e] = 0;
    if (e == 0 && range_dst) *range_dst = range;
  }
  if (bad_ev) return;
  if (hist)
    for (int32_t b = i; b < n_bins; b += stride) hist[int64_t(e) * vw.hist_stride + b] = 0u;
  if (lbh)
    for (int32_t b = i; b < n_bins; b += stride) lbh[int64_t(e) * vw.hist_stride + b] = 0u;
  if (tlb)
    for (int64_t t = i; t < vw.tri_stride; t += stride) {
      tlb[int64_t(e) * vw.tri_stride + t] = 0;
      tn2[int64_t(e) * vw.tri_stride + t] = 0;
    }
  for (int32_t h = i; h < n_hits; h += stride) {
    bool bad;
    prep_one(hits + 8 * static_cast<int64_t>(beg + h), active ? active[beg + h] != 0 : true, &out[beg + h], &bad,
             xr, yr);
    if (assigned) assigned[beg + h] = -1;
    if (bad) {
      atomicOr(status, kStBadHit);
      atomicAdd(reinterpret_cast<unsigned long long*>(n_bad), 1ull);
    }
  }
}

// ---------------------------------------------------------------------------
// top-k selection by (votes desc, index asc).
// threshold v*: the largest v with count(votes >= v) >= k_eff; every box above
// v* is taken, and the first (k_eff - count(votes > v*)) boxes at v* in index
// order (prefix-sum compaction over the chunks of the grid).
struct SelInfo { int32_t vstar, need_eq, n_gt, k_eff; };

IA_HD SelInfo threshold(const uint32_t* hist, int32_t n_bins, int32_t k, uint32_t n_boxes) {
  SelInfo s;
  s.k_eff = static_cast<int32_t>(min(static_cast<uint32_t>(k), n_boxes));
  int64_t cum = 0;
  s.vstar = 0;
  s.need_eq = s.k_eff;
  for (int32_t v = n_bins - 1; v >= 0; --v) {
    const int64_t c = hist[v];
    if (cum + c >= s.k_eff) { s.vstar = v; s.need_eq = static_cast<int32_t>(s.k_eff - cum); break; }
    cum += c;
  }
  s.n_gt = s.k_eff - s.need_eq;
  return s;
}

// block-wide exclusive scan of 0/1 flags (kWG lanes); returns the total
__device__ __forceinline__ int32_t block_scan(int32_t flag, int32_t* excl, int32_t* sbuf) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag != 0);
  const int32_t before = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) sbuf[wv] = __popcll(m);
  __syncthreads();
  int32_t off = 0, tot = 0;
  for (int w = 0; w < kWG / 64; ++w) { if (w < wv) off += sbuf[w]; tot += sbuf[w]; }
  __syncthreads();
  *excl = off + before;
  return tot;
}

// block-wide exclusive scan of non-negative counts (kWG lanes); returns the total
__device__ __forceinline__ int32_t block_scan_count(int32_t v, int32_t* excl, int32_t* sbuf) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sbuf[wv] = x;
  __syncthreads();
  int32_t off = 0, tot = 0;
  for (int w = 0; w < kWG / 64; ++w) { if (w < wv) off += sbuf[w]; tot += sbuf[w]; }
  __syncthreads();
  *excl = off + x - v;
  return tot;
}

__device__ __forceinline__ int32_t block_sum(int32_t v, int32_t* sbuf) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sbuf[threadIdx.x >> 6] = v;
  __syncthreads();
  int32_t t = 0;
  for (int w = 0; w < kWG / 64; ++w) t += sbuf[w];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// Classes of every (triple, hit) pair of a level, and vote bounds per triple.
// class 0: no box of the triple gets the hit's vote; 1: every box does;
// 2: the boxes must be evaluated (stereo hits only).  Axial pairs are decided
// here completely.  With `filter` off every well-formed stereo pair is class
// 2.  With pflags (refinement levels), a hit the parent-level test excluded
// is class 0 for every triple of that parent.  Per triple: tlb = number of class-1 pairs (a lower bound of each of
// its boxes' votes, exact for a triple without class-2 pairs), tn2 = number
// of class-2 pairs (tlb + tn2 bounds the votes from above); both are added
// to (they start at zero).
// Thread = triple: a workgroup takes 64 consecutive triples; its four waves
// and the gridDim.z workgroups of a triple group share the hits (wave w of
// group z takes hits 4 z + w, 4 z + w + 4 gridDim.z, ...), so the hit of a
// wave is uniform (axial and stereo work do not diverge) and each thread
// computes its triple frame once.  flags are hit-major: flags[h * n_tr + t].
// A stereo pair the quick stage leaves undecided gets a deferred flag
// (kFlagDeferred .. kFlagDeferred + 2, with its open drift signs) and is
// classified by k_classify_defer, which must run next: the enclosure passes
// run there on compacted pairs, so that the lanes of a wave whose pairs were
// decided here do not wait for them.
// With COUNT, the work done (residuals G, axial tests, pair quantities,
// magnitude bounds; live triples only) is added to `work` with one atomic
// per counter per workgroup (a separate instantiation: the counting costs
// the search a few per cent).
// Waves per SIMD: 5 at FP64 (at most 96 VGPRs, with eight 8-byte spills in
// the hit loop; 5 % faster than 4 waves at 113 VGPRs), 4 at FP32.
template <bool F32, bool COUNT>
__global__ void __launch_bounds__(kWG, F32 ? 4 : 5) k_classify(const HitRec* __restrict__ hits, EvView vw,
                                                  const BoxD* __restrict__ parents, Shape sh,
                                                  uint8_t* __restrict__ flags, int32_t* __restrict__ tlb,
                                                  int32_t* __restrict__ tn2, int32_t filter,
                                                  const EventState* __restrict__ ev, float slack32,
                                                  const uint8_t* __restrict__ pflags,
                                                  const ParentE* __restrict__ pe,
                                                  unsigned long long* __restrict__ work) {
  const int e = blockIdx.y;
  if (ev && ev[e].done) return;
  const int32_t n_hits = vw.count(e);
  hits += vw.beg(e);
  parents += e * vw.par_stride;
  flags += e * vw.flag_stride;
  tlb += e * vw.tri_stride;
  tn2 += e * vw.tri_stride;
  const uint32_t n_tr = sh.n_parents * sh.m012;
  const uint32_t lane = threadIdx.x & 63u;
  const int32_t wave = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(threadIdx.x >> 6));
  const uint32_t t = blockIdx.x * 64u + lane;
  const bool live = t < n_tr;
  const uint32_t tq = live ? t : n_tr - 1;
  const uint32_t tc = tq % sh.m012;
  const BoxD& TP = parents[tq / sh.m012];
  const uint8_t* pf = pflags ? pflags + e * vw.pflag_stride + int64_t(tq / sh.m012) * n_hits : nullptr;
  const ParentE* pr = pe ? pe + e * vw.pflag_stride + int64_t(tq / sh.m012) * n_hits : nullptr;
  const Frame f = triple_frame(TP, sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
  Iv Zr, Lr;
  centre_ranges(TP, sh.m, &Zr, &Lr);
  const GTri gt = g_triple(f);
  // the disk condition of the level, once per triple (every hit's pair is
  // class 0 where it fails)
  // with the forward test: about the origin each hit must lie ahead (mode
  // 1); about a moved reference point the origin must lie behind (mode 2)
  const int fwdm = ev ? (vw.fwd ? (ev[e].moved ? 2 : 1) : 0) : vw.fwd;
  const double xr = ev ? ev[e].ref[0] : vw.vref[0], yr = ev ? ev[e].ref[1] : vw.vref[1];
  bool disk_ok = fwdm != 2 || behind_ok(f.Fi, xr, yr);
  if (disk_ok && vw.disk > 0.0) {
    const HitRec dh = disk_hit(xr, yr, vw.disk);
    disk_ok = h_contains0(residual_G(f, dh), f.K, f.sig * dh.d, dh.band);
  }
  int32_t lb = 0, n2 = 0;
  int32_t cw[kCwDefer] = {0, 0, 0, 0, 0};
  const int32_t h_step = static_cast<int32_t>(gridDim.z) * (kWG / 64);
  for (int32_t h = static_cast<int32_t>(blockIdx.z) * (kWG / 64) + wave; h < n_hits; h += h_step) {
    const HitRec hr = hits[h];
    uint8_t fl = 0;
    if (disk_ok && votes_now(hr) && (!pf || pf[h]) && (fwdm != 1 || forward_ok(f.Fi, hr))) {
      const int c = pair_stage1<F32>(f, gt, hr, Zr, Lr, filter, slack32, COUNT ? cw : nullptr, pr ? &pr[h] : nullptr);
      fl = c >= 0 ? static_cast<uint8_t>(c) : defer_flag(-c);
    }
    if (live) flags[int64_t(h) * n_tr + t] = fl;
    lb += fl == 1 ? 1 : 0;
    n2 += fl == 2 ? 1 : 0;
  }
  __shared__ int32_t s_lb[kWG / 64][64], s_n2[kWG / 64][64];
  __shared__ unsigned long long s_cw[kCwDefer];
  if (COUNT && threadIdx.x < kCwDefer) s_cw[threadIdx.x] = 0;
  s_lb[wave][lane] = lb;
  s_n2[wave][lane] = n2;
  __syncthreads();
  if (COUNT && live)
    for (uint32_t k = 0; k < kCwDefer; ++k)
      if (cw[k]) atomicAdd(&s_cw[k], static_cast<unsigned long long>(cw[k]));
  if (wave == 0 && live) {
    int32_t a = 0, b = 0;
    for (int w = 0; w < kWG / 64; ++w) { a += s_lb[w][lane]; b += s_n2[w][lane]; }
    if (a) atomicAdd(&tlb[t], a);
    if (b) atomicAdd(&tn2[t], b);
  }
  if constexpr (COUNT) {
    __syncthreads();
    if (threadIdx.x < kCwDefer && s_cw[threadIdx.x]) {
      unsigned long long* slot =
          work + kWorkSlotU64 * ((blockIdx.x + blockIdx.y * 7u + blockIdx.z * 13u) % kWorkSlots);
      atomicAdd(&slot[kWorkClassify + (F32 ? kCwN : 0) + threadIdx.x], s_cw[threadIdx.x]);
    }
  }
}

// Second stage of the classification: the stereo pairs k_classify deferred.
// A workgroup takes `per` x kWG consecutive flags of one event (thread i
// reads flags i, i + kWG, ...; per <= kDeferPer, smaller for small
// launches so that they still spread over the device), lists the deferred
// ones in LDS with a block scan, and the whole workgroup then works through
// the list, one pair per lane: the triple's frame, G and the pair quantities
// (the same functions and inputs as in k_classify, hence the same values),
// then the per-sign enclosure passes; it writes the class and adds class-1
// and class-2 pairs to the triple's bounds.  Pair indices h * n_tr + t stay
// below 2^32 (the launcher checks).  Waves per SIMD: 4 at FP64 (128 VGPRs,
// no spills), 3 at FP32 (whose enclosures would spill at 128).
constexpr int32_t kDeferPer = 16;
constexpr int32_t kDeferChunk = kDeferPer * kWG;

template <bool F32, bool COUNT>
__global__ void __launch_bounds__(kWG, F32 ? 3 : 4) k_classify_defer(const HitRec* __restrict__ hits, EvView vw,
                                                        const BoxD* __restrict__ parents, Shape sh,
                                                        uint8_t* __restrict__ flags, int32_t* __restrict__ tlb,
                                                        int32_t* __restrict__ tn2, int32_t per,
                                                        const EventState* __restrict__ ev, float slack32,
                                                        unsigned long long* __restrict__ work) {
  const int e = blockIdx.y;
  if (ev && ev[e].done) return;
  const int32_t n_hits = vw.count(e);
  const uint32_t n_tr = sh.n_parents * sh.m012;
  const uint32_t n_pairs = n_tr * static_cast<uint32_t>(n_hits > 0 ? n_hits : 0);
  const uint32_t c0 = blockIdx.x * static_cast<uint32_t>(per * kWG);
  if (c0 >= n_pairs) return;
  hits += vw.beg(e);
  parents += e * vw.par_stride;
  flags += e * vw.flag_stride;
  tlb += e * vw.tri_stride;
  tn2 += e * vw.tri_stride;
  __shared__ uint16_t s_list[kDeferChunk];
  __shared__ int32_t s_scan[kWG];
  uint32_t mask = 0;
  int32_t mine = 0;
#pragma unroll
  for (int k = 0; k < kDeferPer; ++k) {
    const uint32_t p = c0 + static_cast<uint32_t>(k * kWG) + threadIdx.x;
    const bool d = k < per && p < n_pairs && flags[p] >= kFlagDeferred;
    mask |= d ? (1u << k) : 0u;
    mine += d ? 1 : 0;
  }
  int32_t pos;
  const int32_t total = block_scan_count(mine, &pos, s_scan);
#pragma unroll
  for (int k = 0; k < kDeferPer; ++k)
    if (mask & (1u << k)) s_list[pos++] = static_cast<uint16_t>(k * kWG + threadIdx.x);
  __syncthreads();
  int32_t cw[3] = {0, 0, 0};                  // deferred pairs, enclosure passes, inclusion proofs
  for (int32_t i = threadIdx.x; i < total; i += kWG) {
    const uint32_t p = c0 + s_list[i];
    const uint32_t h = p / n_tr, t = p - h * n_tr;
    const uint32_t tc = t % sh.m012;
    const BoxD& TP = parents[t / sh.m012];
    const Frame f = triple_frame(TP, sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
    Iv Zr, Lr;
    centre_ranges(TP, sh.m, &Zr, &Lr);
    const HitRec hr = hits[h];
    const int signs = defer_signs(flags[p]);
    if constexpr (COUNT) ++cw[0];
    const int c = pair_stage2<F32>(f, hr, Zr, Lr, slack32, signs, COUNT ? &cw[1] : nullptr);
    flags[p] = static_cast<uint8_t>(c);
    if (c == 1) atomicAdd(&tlb[t], 1);
    else if (c == 2) atomicAdd(&tn2[t], 1);
  }
  if constexpr (COUNT) {
    __shared__ unsigned long long s_cw[3];
    __syncthreads();
    if (threadIdx.x < 3) s_cw[threadIdx.x] = 0;
    __syncthreads();
    for (int k = 0; k < 3; ++k)
      if (cw[k]) atomicAdd(&s_cw[k], static_cast<unsigned long long>(cw[k]));
    __syncthreads();
    if (threadIdx.x < 3 && s_cw[threadIdx.x]) {
      unsigned long long* slot = work + kWorkSlotU64 * ((blockIdx.x + blockIdx.y * 7u) % kWorkSlots);
      atomicAdd(&slot[kWorkClassify + (F32 ? kCwN : 0) + kCwDefer + threadIdx.x], s_cw[threadIdx.x]);
    }
  }
}

// Parent-level exclusion of a refinement level: pflags[p * n_hits + h] = 0
// when hit h can vote for no child box of parent p (parent_may_vote), else 1.
// With `pe` set, pe[p * n_hits + h] receives the per-sign ranges of d^Ax.
template <bool F32>
__global__ void __launch_bounds__(kWG) k_parent_filter(const HitRec* __restrict__ hits, EvView vw,
                                                       const BoxD* __restrict__ parents, Shape sh,
                                                       uint8_t* __restrict__ pflags, const EventState* __restrict__ ev,
                                                       float slack32, ParentE* __restrict__ pe) {
  const int e = blockIdx.y;
  if (ev[e].done) return;
  const int32_t n_hits = vw.count(e);
  if (n_hits <= 0) return;
  hits += vw.beg(e);
  parents += e * vw.par_stride;
  pflags += e * vw.pflag_stride;
  if (pe) pe += e * vw.pflag_stride;
  const int64_t n = static_cast<int64_t>(sh.n_parents) * n_hits;
  for (int64_t i = int64_t(blockIdx.x) * kWG + threadIdx.x; i < n; i += int64_t(gridDim.x) * kWG) {
    const uint32_t p = static_cast<uint32_t>(i / n_hits);
    const int32_t h = static_cast<int32_t>(i % n_hits);
    pflags[i] = parent_may_vote<F32>(parents[p], sh.m, hits[h], slack32, pe ? &pe[i] : nullptr) ? 1 : 0;
  }
}

// Is a triple evaluated at a level with pruning threshold T and tie cut
// tcut?  Its upper bound must reach T; at T exactly, only triples up to tcut
// (see k_threshold) can hold a selected box.
IA_HD bool triple_live(int32_t lb, int32_t n2, int32_t T, uint32_t t, int32_t tcut) {
  const int32_t ub = lb + n2;
  return ub > T || (ub == T && static_cast<int64_t>(t) <= tcut);
}

// Pruning threshold of a level, one workgroup per event: T = the largest v
// such that at least k_eff = min(k, n_boxes) boxes have a lower bound >= v
// (each triple holds m34 boxes), from the histogram of the triples' lower
// bounds (in LDS, or in lbh -- zero on entry, cleared on exit -- when it has
// more than kHistLds bins); T = 0 without `prune`.  The k_eff-th box of the
// selection has at least T votes, so a triple whose upper bound is below T
// holds no selected box and no box of the maximum.  Then the vote tiles of
// bx boxes holding a triple with upper bound >= T are listed in index order
// (live_list, ev->n_live); the others get wg_max = -1 and are not voted.
// With live_tri, the triples whose class-2 pairs are evaluated (tn2 > 0 and
// upper bound >= T) are listed too (ev->n_live_tri), each with the offset of
// its records (rec_off, in index order; rec_fill cleared); ev->rec_ok tells
// whether all ev->n_rec records fit rec_cap.
// With `ties` (levels whose only use is the top-k selection and the
// maximum, not the estimate's max-vote set): let t_cut be the triple, in
// index order, at which the triples with lower bound >= T first hold k_eff
// boxes.  Those k_eff boxes have at least T votes and lower indices than any
// box after t_cut, so a box after t_cut with at most T votes ranks after all
// of them (votes desc, index asc); a triple after t_cut whose upper bound is
// T is pruned too.  The maximum is unchanged (it is at least T).
// ev->t_cut = INT32_MAX without ties.
//
// Probe (probe = 1, one-box selections, before the level's vote): T is the
// kProbeTriples-th largest upper bound over the triples with class-2 pairs
// (no triple when fewer hold such pairs), cut among the triples at T in index
// order so that kProbeTriples are voted, no drop, and every tile's wg_max is
// set to -1, so that after a vote of the listed tiles (without histogram) the
// largest wg_max is the largest vote v1 found among them, or -1.  After a
// probe (probe = 2): v1 is read from wg_max first, and T = max(T, v1) - drop.
// A box with at least vmax - drop votes has at least max(T, v1) - drop
// (vmax >= T and vmax >= v1), so its triple is still evaluated: selections
// and maxima are those of the plain threshold.
constexpr int32_t kProbeTriples = 8;

__global__ void __launch_bounds__(kWG) k_threshold(const int32_t* __restrict__ tlb, const int32_t* __restrict__ tn2,
                                                   uint32_t* __restrict__ lbh, EvView vw, Shape sh, int32_t k,
                                                   int32_t prune, int32_t ties, int32_t bx, EventState* __restrict__ ev,
                                                   int32_t* __restrict__ live_list, int32_t* __restrict__ wg_max,
                                                   int32_t* __restrict__ live_tri, int32_t* __restrict__ rec_off,
                                                   int32_t* __restrict__ rec_fill, int64_t rec_cap,
                                                   int32_t drop, int32_t probe) {
  const int e = blockIdx.y;
  if (ev[e].done) return;
  const int32_t n_bins = vw.count(e) + 1;
  const uint32_t n_tr = sh.n_parents * sh.m012;
  tlb += e * vw.tri_stride;
  tn2 += e * vw.tri_stride;
  live_list += int64_t(e) * vw.wg_stride;
  wg_max += int64_t(e) * vw.wg_stride;
  __shared__ uint32_t sh_h[kHistLds];
  __shared__ int32_t s_T;
  __shared__ int32_t sbuf[kWG / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t n_tiles = (sh.n_boxes + static_cast<uint32_t>(bx) - 1) / static_cast<uint32_t>(bx);
  int32_t v1 = -1;
  if (prune && probe == 2) {
    // the largest vote the probe found (its tiles' maxima; -1 elsewhere)
    for (uint32_t tile = tid; tile < n_tiles; tile += kWG) v1 = max(v1, wg_max[tile]);
    for (int o = 32; o > 0; o >>= 1) v1 = max(v1, __shfl_down(v1, o, 64));
    if ((tid & 63) == 0) sbuf[tid >> 6] = v1;
    __syncthreads();
    v1 = -1;
    for (int w = 0; w < kWG / 64; ++w) v1 = max(v1, sbuf[w]);
    __syncthreads();
  }
  if (prune) {
    uint32_t* hh = sh_h;
    if (n_bins > kHistLds) hh = lbh + int64_t(e) * vw.hist_stride;
    else
      for (int32_t b = tid; b < n_bins; b += kWG) sh_h[b] = 0u;
    __syncthreads();
    if (probe == 1) {
      for (uint32_t t = tid; t < n_tr; t += kWG)
        if (tn2[t] > 0) atomicAdd(&hh[min(tlb[t] + tn2[t], n_bins - 1)], 1u);
    } else {
      for (uint32_t t = tid; t < n_tr; t += kWG) atomicAdd(&hh[min(tlb[t], n_bins - 1)], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      if (probe == 1) {
        int64_t cum = 0;
        int32_t T = n_bins;               // no triple when fewer than kProbeTriples hold class-2 pairs
        for (int32_t v = n_bins - 1; v >= 0; --v) {
          cum += static_cast<int64_t>(hh[v]);
          if (cum >= kProbeTriples) { T = v; break; }
        }
        s_T = T;
      } else {
        const int64_t k_eff = min(static_cast<int64_t>(k), static_cast<int64_t>(sh.n_boxes));
        int64_t cum = 0;
        int32_t T = 0;
        for (int32_t v = n_bins - 1; v >= 0; --v) {
          cum += static_cast<int64_t>(hh[v]) * sh.m34;
          if (cum >= k_eff) { T = v; break; }
        }
        // drop: boxes down to `drop` votes below the maximum are needed exactly
        s_T = max(max(T, v1) - drop, 0);
      }
    }
    __syncthreads();
    if (n_bins > kHistLds)
      for (int32_t b = tid; b < n_bins; b += kWG) hh[b] = 0u;
  } else if (tid == 0) {
    s_T = 0;
  }
  __syncthreads();
  const int32_t T = s_T;
  __shared__ int32_t s_cut;
  if (tid == 0) s_cut = INT32_MAX;
  __syncthreads();
  if (prune && ties) {
    // t_cut: the triple at which the boxes of triples with lower bound >= T
    // reach k_eff, in index order (contiguous runs of triples per thread)
    const int64_t k_eff = min(static_cast<int64_t>(k), static_cast<int64_t>(sh.n_boxes));
    const uint32_t pt = (n_tr + kWG - 1) / kWG;
    const uint32_t ra = min(tid * pt, n_tr), rb = min(ra + pt, n_tr);
    int32_t c = 0;
    for (uint32_t t = ra; t < rb; ++t) c += tlb[t] >= T ? 1 : 0;
    int32_t before;
    block_scan_count(c, &before, sbuf);
    int64_t cum = static_cast<int64_t>(before) * sh.m34;
    if (cum < k_eff && cum + static_cast<int64_t>(c) * sh.m34 >= k_eff) {
      for (uint32_t t = ra; t < rb; ++t) {
        if (tlb[t] < T) continue;
        cum += sh.m34;
        if (cum >= k_eff) { s_cut = static_cast<int32_t>(t); break; }
      }
    }
    __syncthreads();
  }
  if (prune && probe == 1 && T < n_bins) {
    // the probe's tie cut: exactly kProbeTriples triples with class-2 pairs,
    // those whose upper bound is above T, then those at T in index order
    const uint32_t pt = (n_tr + kWG - 1) / kWG;
    const uint32_t ra = min(tid * pt, n_tr), rb = min(ra + pt, n_tr);
    int32_t ca = 0, ct = 0;
    for (uint32_t t = ra; t < rb; ++t)
      if (tn2[t] > 0) {
        const int32_t ub = tlb[t] + tn2[t];
        ca += ub > T ? 1 : 0;
        ct += ub == T ? 1 : 0;
      }
    int32_t ba, bt;
    const int32_t n_above = block_scan_count(ca, &ba, sbuf);
    block_scan_count(ct, &bt, sbuf);
    const int32_t need = kProbeTriples - n_above;   // >= 1: fewer than kProbeTriples lie above T
    if (bt < need && bt + ct >= need) {
      int32_t cum = bt;
      for (uint32_t t = ra; t < rb; ++t) {
        if (tn2[t] == 0 || tlb[t] + tn2[t] != T) continue;
        if (++cum == need) { s_cut = static_cast<int32_t>(t); break; }
      }
    }
    __syncthreads();
  }
  const int32_t tcut = s_cut;
  // live tiles, compacted in index order: each thread takes a contiguous run
  // of tiles, counts its live ones, and one block scan places them
  auto triple_of = [&](uint32_t x) { return (x / sh.nc) * sh.m012 + (x % sh.nc) / sh.m34; };
  const uint32_t per = (n_tiles + kWG - 1) / kWG;
  const uint32_t ta = min(tid * per, n_tiles), tb = min(ta + per, n_tiles);
  auto tile_live = [&](uint32_t tile) {
    const uint32_t b0 = tile * static_cast<uint32_t>(bx);
    const uint32_t b1 = min(b0 + static_cast<uint32_t>(bx), sh.n_boxes) - 1;
    bool lv = false;
    for (uint32_t t = triple_of(b0); t <= triple_of(b1) && !lv; ++t) lv = triple_live(tlb[t], tn2[t], T, t, tcut);
    return lv;
  };
  // the first 32 tiles' liveness is kept in a bit mask for the second pass
  int32_t mine = 0;
  uint32_t lmask = 0;
  for (uint32_t tile = ta; tile < tb; ++tile) {
    const bool lv = tile_live(tile);
    if (lv) {
      ++mine;
      if (tile - ta < 32u) lmask |= 1u << (tile - ta);
    }
    if (!lv || probe == 1) wg_max[tile] = -1;
  }
  int32_t pos;
  const int32_t total = block_scan_count(mine, &pos, sbuf);
  for (uint32_t tile = ta; tile < tb; ++tile)
    if (tile - ta < 32u ? ((lmask >> (tile - ta)) & 1u) != 0u : tile_live(tile))
      live_list[pos++] = static_cast<int32_t>(tile);
  int32_t n_lt = 0, n_rec = 0;
  if (live_tri) {
    // triples whose class-2 pairs are evaluated, and their record offsets
    live_tri += e * vw.tri_stride;
    rec_off += e * vw.tri_stride;
    rec_fill += e * vw.tri_stride;
    const uint32_t pt = (n_tr + kWG - 1) / kWG;
    const uint32_t ra = min(tid * pt, n_tr), rb = min(ra + pt, n_tr);
    int32_t c1 = 0, c2 = 0;
    for (uint32_t t = ra; t < rb; ++t)
      if (tn2[t] > 0 && triple_live(tlb[t], tn2[t], T, t, tcut)) { ++c1; c2 += tn2[t]; }
    int32_t p1, p2;
    n_lt = block_scan_count(c1, &p1, sbuf);
    n_rec = block_scan_count(c2, &p2, sbuf);
    for (uint32_t t = ra; t < rb; ++t)
      if (tn2[t] > 0 && triple_live(tlb[t], tn2[t], T, t, tcut)) {
        live_tri[p1++] = static_cast<int32_t>(t);
        rec_off[t] = p2;
        rec_fill[t] = 0;
        p2 += tn2[t];
      }
  }
  if (tid == 0) {
    ev[e].t_prune = T;
    ev[e].t_cut = tcut;
    ev[e].n_live = total;
    ev[e].n_live_tri = n_lt;
    ev[e].n_rec = n_rec;
    ev[e].rec_ok = live_tri != nullptr && static_cast<int64_t>(n_rec) <= rec_cap ? 1 : 0;
  }
}

// Staged records of a level.  Items are (hit, listed triple) pairs; a
// workgroup takes kStageBatch x kWG consecutive items, keeps the class-2
// ones in an LDS list (most pairs are decided, so computing in place would
// leave most lanes of a wave idle), then computes one record per listed
// pair with all its lanes: the triple's frame, G and the pair quantities
// (FP64, or their FP32 images at FP32 levels), written with the hit's
// tan(tau), drift and band to a slot of its triple's record range (slots
// taken in any order: votes do not depend on it).  Every writer of a triple
// also writes the same TriFrame.  Events with rec_ok == 0 are skipped.
constexpr int kStageBatch = 4;

template <bool F32>
__global__ void __launch_bounds__(kWG, 4) k_stage(const HitRec* __restrict__ hits_all, EvView vw,
                                               const BoxD* __restrict__ parents_all, Shape sh,
                                               const uint8_t* __restrict__ flags_all,
                                               const int32_t* __restrict__ live_tri_all,
                                               const int32_t* __restrict__ rec_off_all,
                                               int32_t* __restrict__ rec_fill_all, void* __restrict__ rec,
                                               TriFrame* __restrict__ tfr_all, const int64_t* __restrict__ stage_off,
                                               int32_t n_ev, float slack32) {
  const uint32_t n_tr = sh.n_parents * sh.m012;
  const int64_t n_items = stage_off[n_ev];
  __shared__ int64_t slist[kStageBatch * kWG];
  __shared__ int32_t sev[kStageBatch * kWG];
  __shared__ int32_t scount;
  const int64_t span = int64_t(kStageBatch) * kWG;
  for (int64_t base = int64_t(blockIdx.x) * span; base < n_items; base += int64_t(gridDim.x) * span) {
    if (threadIdx.x == 0) scount = 0;
    // the event of the batch's first item: the last one whose first item is
    // at or before it (the same for every thread); later items step forward
    int32_t e_base = 0;
    {
      int32_t elo = 0, ehi = n_ev - 1;
      while (elo < ehi) {
        const int32_t mid = (elo + ehi + 1) >> 1;
        if (stage_off[mid] <= base) elo = mid;
        else ehi = mid - 1;
      }
      e_base = elo;
    }
    __syncthreads();
    int32_t e = e_base;
    for (int r = 0; r < kStageBatch; ++r) {
      const int64_t i = base + int64_t(r) * kWG + threadIdx.x;
      bool keep = false;
      if (i < n_items) {
        while (e + 1 < n_ev && stage_off[e + 1] <= i) ++e;
        // hit-major within the event: neighbouring lanes read neighbouring
        // live triples' flags of one hit (flags are [hit][triple])
        const int64_t n_lt = (stage_off[e + 1] - stage_off[e]) / vw.count(e);
        const int64_t il = i - stage_off[e];
        const uint32_t t = static_cast<uint32_t>(live_tri_all[e * vw.tri_stride + il % n_lt]);
        const int32_t h = static_cast<int32_t>(il / n_lt);
        keep = flags_all[e * vw.flag_stride + int64_t(h) * n_tr + t] == 2;
      }
      // wave-level compaction: one LDS atomic per wave
      const unsigned long long m = __ballot(keep);
      const uint32_t lane = threadIdx.x & 63u;
      int32_t wbase = 0;
      if (lane == 0 && m) wbase = atomicAdd(&scount, __popcll(m));
      wbase = __shfl(wbase, 0, 64);
      if (keep) {
        const int32_t pos = wbase + __popcll(m & ((1ull << lane) - 1ull));
        slist[pos] = i;
        sev[pos] = e;
      }
    }
    __syncthreads();
    const int32_t n = scount;
    for (int32_t j = threadIdx.x; j < n; j += kWG) {
      const int64_t i = slist[j];
      const int e = sev[j];
      const int64_t n_lt = (stage_off[e + 1] - stage_off[e]) / vw.count(e);
      const int64_t il = i - stage_off[e];
      const HitRec* hits = hits_all + vw.beg(e);
      const BoxD* parents = parents_all + e * vw.par_stride;
      const int32_t* rec_off = rec_off_all + e * vw.tri_stride;
      int32_t* rec_fill = rec_fill_all + e * vw.tri_stride;
      TriFrame* tfr = tfr_all + e * vw.tri_stride;
      const uint32_t t = static_cast<uint32_t>(live_tri_all[e * vw.tri_stride + il % n_lt]);
      const int32_t h = static_cast<int32_t>(il / n_lt);
      const HitRec hr = hits[h];
      const uint32_t tc = t % sh.m012;
      const Frame f = triple_frame(parents[t / sh.m012], sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
      const int64_t slot = int64_t(e) * vw.rec_stride + rec_off[t] + atomicAdd(&rec_fill[t], 1);
      if constexpr (F32) {
        const Frame32 g32 = frame32_of(f);
        reinterpret_cast<PairQ32*>(rec)[slot] = pair_q32_f32(g32, hr, slack32);
        tfr[t] = TriFrame{static_cast<double>(g32.R), static_cast<double>(g32.sig), f.K.lo, f.K.hi};
      } else {
        const Iv G = residual_G(f, hr);
        const PairQ q = pair_quantities(f, hr, G);
        RecD r;
        r.q[0] = q.Glo; r.q[1] = q.Ghi; r.q[2] = q.sArc; r.q[3] = q.dphi; r.q[4] = q.RAx; r.q[5] = q.sinA;
        r.q[6] = q.cosA; r.q[7] = q.sAx; r.q[8] = q.cAx; r.q[9] = q.c2; r.q[10] = q.s2; r.q[11] = q.twoRAx2;
        r.q[12] = q.RpRAx;
        r.tt = hr.tant;
        r.d = hr.d;
        r.band = hr.band;
        reinterpret_cast<RecD*>(rec)[slot] = r;
        tfr[t] = TriFrame{f.R, f.sig, f.K.lo, f.K.hi};
      }
    }
    __syncthreads();                     // the list is rebuilt for the next batch
  }
}

// Top-k by (votes desc, index asc) of one level, one workgroup, run after
// the vote kernel has written the votes, the histogram and the maximum of
// each of its n_wg workgroups (bx boxes each).  Boxes above the threshold v*
// or at it can only sit in workgroups whose maximum reaches v*; those are
// visited in index order, kWG / bx at a time, and compacted with block scans
// until all count(> v*) boxes and the first (k - count(> v*)) boxes at v*
// are collected (at most k workgroups hold boxes above v*).  Then the entries
// are ordered, the selected boxes written, the histogram cleared and, for
// level 0, the event stopped when its maximum is below v_min.  k <= vw.k
// boxes are selected (vw.k is the per-event stride of the outputs); the
// histogram must count at least min(k, n_boxes) boxes.
__global__ void __launch_bounds__(kWG) k_select_wg(const uint16_t* __restrict__ votes, EvView vw,
                                                   uint32_t* __restrict__ hist, const int32_t* __restrict__ wg_max,
                                                   uint32_t n_wg, int32_t bx, const BoxD* __restrict__ parents,
                                                   Shape sh, BoxD* __restrict__ out_boxes,
                                                   int64_t* __restrict__ out_index, uint16_t* __restrict__ out_votes,
                                                   EventState* __restrict__ ev, int32_t v_min_stop,
                                                   int32_t* __restrict__ tlb, int32_t* __restrict__ tn2, int32_t k) {
  const int e = blockIdx.y;
  if (ev && ev[e].done) return;
  const uint32_t n_boxes = sh.n_boxes;
  const int32_t n_bins = vw.count(e) + 1;
  votes += int64_t(e) * n_boxes;
  hist += int64_t(e) * vw.hist_stride;
  wg_max += int64_t(e) * vw.wg_stride;
  parents += e * vw.par_stride;
  out_boxes += int64_t(e) * vw.k;
  out_index += int64_t(e) * vw.k;
  out_votes += int64_t(e) * vw.k;
  if (ev) ev += e;
  __shared__ SelInfo si;
  __shared__ int32_t sbuf[kWG / 64];
  __shared__ int32_t s_vmax, s_run_gt, s_run_eq;
  __shared__ uint32_t s_nmax;
  __shared__ uint32_t s_idx[kMaxTopK];
  __shared__ uint16_t s_v[kMaxTopK];
  __shared__ uint32_t s_list[kWG];
  const int tid = threadIdx.x;
  if (tid == 0) {
    si = threshold(hist, n_bins, k, n_boxes);
    int32_t vm = 0;
    uint32_t nm = 0;
    for (int32_t v = n_bins - 1; v >= 0; --v) {
      const uint32_t c = hist[v];
      if (c != 0u) { vm = v; nm = c; break; }
    }
    s_vmax = vm;
    s_nmax = nm;
    s_run_gt = 0;
    s_run_eq = 0;
  }
  __syncthreads();
  const int32_t per = max(1, kWG / bx);            // candidate workgroups per pass
  for (uint32_t w0 = 0; w0 < n_wg; w0 += kWG) {
    if (s_run_gt >= si.n_gt && s_run_eq >= si.need_eq) break;
    const uint32_t w = w0 + tid;
    const int32_t m = w < n_wg ? wg_max[w] : -1;
    const int32_t cand = (m > si.vstar) || (m == si.vstar && s_run_eq < si.need_eq);
    int32_t xc;
    const int32_t nc = block_scan(cand, &xc, sbuf);
    if (cand) s_list[xc] = w;
    __syncthreads();
    for (int32_t c0 = 0; c0 < nc; c0 += per) {
      if (s_run_gt >= si.n_gt && s_run_eq >= si.need_eq) break;
      // thread -> (candidate c0 + tid / bx, box tid % bx): index order is thread order
      const int32_t ci = c0 + tid / bx;
      const bool ok = tid < per * bx && ci < nc;
      const uint32_t b = ok ? s_list[ci] * static_cast<uint32_t>(bx) + static_cast<uint32_t>(tid % bx) : 0u;
      const int32_t v = (ok && b < n_boxes) ? static_cast<int32_t>(votes[b]) : -1;
      const int32_t fg = v > si.vstar, fe = v == si.vstar;
      int32_t xg, xe;
      const int32_t run_gt = s_run_gt, run_eq = s_run_eq;
      const int32_t tg = block_scan(fg, &xg, sbuf);
      const int32_t te = block_scan(fe, &xe, sbuf);
      if (fg && run_gt + xg < si.n_gt) s_idx[run_gt + xg] = b;
      if (fe && run_eq + xe < si.need_eq) s_idx[si.n_gt + run_eq + xe] = b;
      __syncthreads();
      if (tid == 0) { s_run_gt = run_gt + tg; s_run_eq = run_eq + te; }
      __syncthreads();
    }
  }
  const int32_t ke = si.k_eff;
  for (int32_t a = tid; a < ke; a += kWG) s_v[a] = votes[s_idx[a]];
  __syncthreads();
  for (int32_t a = tid; a < ke; a += kWG) {
    const uint32_t ia = s_idx[a];
    const int32_t va = s_v[a];
    int32_t rank = 0;
    for (int32_t c = 0; c < ke; ++c) {
      const int32_t vc = s_v[c];
      rank += (vc > va) || (vc == va && s_idx[c] < ia);
    }
    out_index[rank] = ia;
    out_votes[rank] = static_cast<uint16_t>(va);
    level_box(parents, sh, ia, &out_boxes[rank]);
  }
  __syncthreads();
  for (int32_t i = tid; i < n_bins; i += kWG) hist[i] = 0u;
  if (tlb) {
    // the level's triple bounds start at zero for the next classification
    const uint32_t n_tr = sh.n_parents * sh.m012;
    tlb += e * vw.tri_stride;
    tn2 += e * vw.tri_stride;
    for (uint32_t t = tid; t < n_tr; t += kWG) { tlb[t] = 0; tn2[t] = 0; }
  }
  if (tid == 0 && ev) {
    ev->vmax = s_vmax;
    ev->n_argmax = static_cast<int32_t>(s_nmax);
    ev->k_sel = ke;
    if (v_min_stop > 0 && s_vmax < v_min_stop) ev->done = 1;
  }
}

// ---------------------------------------------------------------------------
// the vote kernel.  The boxes of a level form tiles of BX consecutive boxes;
// a workgroup takes one tile at a time (one box per lane), striding over the
// event's live tiles (live_list[0 .. ev->n_live), from k_threshold) or, with
// live_list null, over every tile.  Within a tile it splits each hit chunk
// over kWG / BX slices (whole waves) whose counts are summed in LDS.  Each
// box starts from its triple's lower bound tlb (its class-1 pairs from
// k_classify, axial ones included); class-2 pairs are evaluated per box only
// in triples whose upper bound tlb + tn2 reaches the event's pruning
// threshold T (ev->t_prune, 0 without ev).  Per chunk of hits, the workgroup
// stages the (triple, hit) quantities of those pairs in LDS.
// Writes the votes of its tiles, each tile's maximum (wg_max) and, with
// hist, the histogram of the votes >= T (the selection threshold is never
// below T).  Tiles that are not live are neither written nor counted.
// With only_unstaged, it votes only the events whose records did not fit
// (k_vote_rec votes the others).
template <int BX, bool F32, bool EXACT = false>
__global__ void __launch_bounds__(kWG) k_vote(const HitRec* __restrict__ hits, EvView vw,
                                              const BoxD* __restrict__ parents, Shape sh,
                                              uint16_t* __restrict__ votes, uint32_t* __restrict__ hist,
                                              uint32_t* __restrict__ status, const EventState* __restrict__ ev,
                                              const uint8_t* __restrict__ flags, const int32_t* __restrict__ tlb,
                                              const int32_t* __restrict__ tn2, const int32_t* __restrict__ live_list,
                                              int32_t* __restrict__ wg_max, unsigned long long* __restrict__ work,
                                              float slack32, int32_t only_unstaged) {
  constexpr int HS = kWG / BX;
  static_assert(BX % 64 == 0 && HS * BX == kWG, "slices are whole waves");
  const int e = blockIdx.y;
  if (ev && ev[e].done) return;
  if (only_unstaged && ev[e].rec_ok) return;   // k_vote_rec covers this event
  const int32_t n_hits = vw.count(e), n_bins = n_hits + 1;
  hits += vw.beg(e);
  parents += e * vw.par_stride;
  votes += int64_t(e) * sh.n_boxes;
  if (hist) hist += int64_t(e) * vw.hist_stride;
  flags += e * vw.flag_stride;
  tlb += e * vw.tri_stride;
  tn2 += e * vw.tri_stride;
  if (wg_max) wg_max += int64_t(e) * vw.wg_stride;
  if (live_list) live_list += int64_t(e) * vw.wg_stride;
  const int32_t T = ev ? ev[e].t_prune : 0;
  const int32_t tcut = ev ? ev[e].t_cut : INT32_MAX;
  const uint32_t n_tr = sh.n_parents * sh.m012;
  const uint32_t n_tiles = (sh.n_boxes + BX - 1) / BX;
  const uint32_t n_items = live_list ? static_cast<uint32_t>(ev[e].n_live) : n_tiles;
  __shared__ double sq[14][kCap + 16];
  // FP32 levels stage 16 floats per pair in the same storage
  static_assert(sizeof(PairQ32) == 16 * sizeof(float) && 16 * 4 <= 14 * 8, "FP32 staging fits");
  float(*sq32)[kCap + 16] = reinterpret_cast<float(*)[kCap + 16]>(&sq[0][0]);
  __shared__ int8_t sflag[kCap + 16];
  __shared__ int8_t stlive[kWG];
  __shared__ uint32_t shist[kHistLds];
  __shared__ int32_t sred[HS][BX];
  __shared__ int32_t sbuf[kWG / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t bl = tid % BX, sl = tid / BX;
  // global triple index of a box: parent * m012 + (child / m34)
  auto triple_of = [&](uint32_t x) { return (x / sh.nc) * sh.m012 + (x % sh.nc) / sh.m34; };
  int32_t n_eval = 0, n_staged = 0;

  for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const uint32_t tile = live_list ? static_cast<uint32_t>(live_list[item]) : item;
    const uint32_t b0 = tile * BX;
    const uint32_t b_last = min(b0 + BX, sh.n_boxes) - 1;
    const uint32_t b = b0 + bl;
    const bool live = b < sh.n_boxes;
    const uint32_t bb = live ? b : b_last;
    const uint32_t t_first = triple_of(b0);
    const int32_t nt = static_cast<int32_t>(triple_of(b_last) - t_first + 1);
    const int32_t my_tl = static_cast<int32_t>(triple_of(bb) - t_first);
    const int32_t hc = max(1, kCap / nt);          // hits per chunk
    // LDS row pitch per triple: one padding slot when a few triples share a
    // wave (avoids bank conflicts); nt * pitch <= kCap + 16 always holds.
    const int32_t pitch = hc + ((nt > 1 && nt <= 16) ? 1 : 0);

    __syncthreads();                     // LDS of the previous tile is free
    // triples of this tile that need per-box evaluation
    int32_t any_live = 0;
    for (int32_t i = tid; i < nt; i += kWG) {
      const int32_t a = tlb[t_first + i], c = tn2[t_first + i];
      const bool lv = c > 0 && triple_live(a, c, T, t_first + i, tcut);
      stlive[i] = lv ? 1 : 0;
      any_live |= lv ? 1 : 0;
    }
    any_live = __syncthreads_or(any_live);

    int32_t nv = sl == 0 ? tlb[t_first + my_tl] : 0;
    if (any_live) {                      // uniform over the workgroup (barriers below)
      // this lane's box: triple frame and (z0, tanl) centre
      uint32_t k[5];
      child_index(sh.m, bb % sh.nc, k);
      const BoxD& P = parents[bb / sh.nc];
      const Frame f = triple_frame(P, sh.m, k[0], k[1], k[2]);
      double zlo, zhi, llo, lhi;
      child_edge(P.lo[3], P.hi[3], sh.m[3], k[3], &zlo, &zhi);
      child_edge(P.lo[4], P.hi[4], sh.m[4], k[4], &llo, &lhi);
      const double z0 = 0.5 * (zlo + zhi), lam = 0.5 * (llo + lhi);
      const double lamR = lam * f.R, lam2 = lam * lam;
      // FP32 images of the lane's box (used at FP32 levels only): the FP32
      // frame's radius and sign, kappa rounded outward
      float R32 = 0.0f, sig32 = 0.0f;
      if constexpr (F32) {
        const Frame32 g32 = frame32_of(f);
        R32 = g32.R;
        sig32 = g32.sig;
      }
      const Iv32 K32 = to32(f.K);
      const float z032 = static_cast<float>(z0), lam32 = static_cast<float>(lam);
      const float lamR32 = lam32 * R32, lam232 = lam32 * lam32;

      for (int32_t h0 = 0; h0 < n_hits; h0 += hc) {
        const int32_t nh = min(hc, n_hits - h0);
        __syncthreads();
        // stage the class-2 pairs of live triples: thread r -> (tl = r / hc, hl = r % hc)
        for (int32_t r = tid; r < nt * hc; r += kWG) {
          const int32_t tl = r / hc, hl = r % hc;
          const int32_t slot = tl * pitch + hl;
          if (hl >= nh) continue;
          const uint32_t t = t_first + tl;
          if (!stlive[tl] || flags[int64_t(h0 + hl) * n_tr + t] != 2) { sflag[slot] = 0; continue; }
          const HitRec h = hits[h0 + hl];
          const uint32_t tc = t % sh.m012;
          const uint32_t t0 = tc / sh.m12, t1 = (tc / sh.m[2]) % sh.m[1], t2 = tc % sh.m[2];
          const Frame ft = triple_frame(parents[t / sh.m012], sh.m, t0, t1, t2);
          ++n_staged;
          sflag[slot] = 2;
          if constexpr (F32) {
            const PairQ32 rq = pair_q32_f32(frame32_of(ft), h, slack32);
            sq32[0][slot] = rq.Glo; sq32[1][slot] = rq.Ghi; sq32[2][slot] = rq.sArc; sq32[3][slot] = rq.dphi;
            sq32[4][slot] = rq.RAx; sq32[5][slot] = rq.sinA; sq32[6][slot] = rq.cosA; sq32[7][slot] = rq.sAx;
            sq32[8][slot] = rq.cAx; sq32[9][slot] = rq.c2; sq32[10][slot] = rq.s2; sq32[11][slot] = rq.twoRAx2;
            sq32[12][slot] = rq.RpRAx; sq32[13][slot] = rq.tt; sq32[14][slot] = rq.d; sq32[15][slot] = rq.bs;
          } else {
            const Iv G = residual_G(ft, h);
            const PairQ q = pair_quantities(ft, h, G);
            sq[0][slot] = q.Glo; sq[1][slot] = q.Ghi; sq[2][slot] = q.sArc; sq[3][slot] = q.dphi;
            sq[4][slot] = q.RAx; sq[5][slot] = q.sinA; sq[6][slot] = q.cosA; sq[7][slot] = q.sAx;
            sq[8][slot] = q.cAx; sq[9][slot] = q.c2; sq[10][slot] = q.s2; sq[11][slot] = q.twoRAx2;
            sq[12][slot] = q.rRAx; sq[13][slot] = q.r2RAx2;
          }
        }
        __syncthreads();
        if (!stlive[my_tl]) continue;
        for (int32_t hl = sl; hl < nh; hl += HS) {
          const int32_t slot = my_tl * pitch + hl;
          if (sflag[slot] != 2) continue;
          n_eval += live ? 1 : 0;
          if constexpr (F32) {
            PairQ32 r;
            r.Glo = sq32[0][slot]; r.Ghi = sq32[1][slot]; r.sArc = sq32[2][slot]; r.dphi = sq32[3][slot];
            r.RAx = sq32[4][slot]; r.sinA = sq32[5][slot]; r.cosA = sq32[6][slot]; r.sAx = sq32[7][slot];
            r.cAx = sq32[8][slot]; r.c2 = sq32[9][slot]; r.s2 = sq32[10][slot]; r.twoRAx2 = sq32[11][slot];
            r.RpRAx = sq32[12][slot]; r.tt = sq32[13][slot]; r.d = sq32[14][slot]; r.bs = sq32[15][slot];
            if (stereo_vote32(r, R32, sig32, K32, z032, lam32, lamR32, lam232)) ++nv;
          } else {
            const HitRec& h = hits[h0 + hl];
            PairQ q;
            q.Glo = sq[0][slot]; q.Ghi = sq[1][slot]; q.sArc = sq[2][slot]; q.dphi = sq[3][slot];
            q.RAx = sq[4][slot]; q.sinA = sq[5][slot]; q.cosA = sq[6][slot]; q.sAx = sq[7][slot];
            q.cAx = sq[8][slot]; q.c2 = sq[9][slot]; q.s2 = sq[10][slot]; q.twoRAx2 = sq[11][slot];
            q.rRAx = sq[12][slot]; q.r2RAx2 = sq[13][slot];
            q.RpRAx = f.R + q.RAx;             // as pair_quantities forms it, same frame
            const double tt = h.tant;
            if (stereo_vote<EXACT>(q, f.R, f.sig, f.K, z0, lam, lamR, lam2, tt, tt * tt, h.d, h.band)) ++nv;
          }
        }
      }
    }
    if (HS > 1) {
      __syncthreads();
      sred[sl][bl] = nv;
      __syncthreads();
      if (sl == 0)
        for (int s = 1; s < HS; ++s) nv += sred[s][bl];
    }
    const bool owner = sl == 0 && live;
    if (owner) votes[b] = static_cast<uint16_t>(nv);
    // tile maximum (read by the selection kernel and used below)
    int32_t mv = owner ? nv : -1;
    for (int o = 32; o > 0; o >>= 1) mv = max(mv, __shfl_down(mv, o, 64));
    __syncthreads();
    if ((tid & 63) == 0) sbuf[tid >> 6] = mv;
    __syncthreads();
    int32_t wmax = -1;
    for (int w = 0; w < kWG / 64; ++w) wmax = max(wmax, sbuf[w]);
    if (wg_max && tid == 0) wg_max[tile] = wmax;
    // vote histogram of the bins >= T; nothing to add when the maximum is below
    if (hist && wmax >= T) {
      const bool in_lds = n_bins <= kHistLds;
      if (in_lds) {
        for (int32_t i = tid; i < n_bins; i += kWG) shist[i] = 0u;
        __syncthreads();
      }
      if (owner && nv >= T) {
        if (nv >= n_bins) atomicOr(status, kStVoteOverflow);
        else if (in_lds) atomicAdd(&shist[nv], 1u);
        else atomicAdd(&hist[nv], 1u);
      }
      if (in_lds) {
        __syncthreads();
        for (int32_t i = tid; i < n_bins; i += kWG)
          if (shist[i]) atomicAdd(&hist[i], shist[i]);
      }
    }
  }
  if (work) {
    // work done by this workgroup: summed over its waves in LDS, then one
    // atomic per counter into one of kWorkSlots cache-line-sized slots
    int32_t a = n_eval, b2 = n_staged;
    for (int o = 32; o > 0; o >>= 1) { a += __shfl_down(a, o, 64); b2 += __shfl_down(b2, o, 64); }
    __shared__ int32_t swork[2][kWG / 64];
    __syncthreads();
    if ((tid & 63) == 0) { swork[0][tid >> 6] = a; swork[1][tid >> 6] = b2; }
    __syncthreads();
    if (tid == 0) {
      int32_t sa = 0, sb = 0;
      for (int w = 0; w < kWG / 64; ++w) { sa += swork[0][w]; sb += swork[1][w]; }
      unsigned long long* slot = work + kWorkSlotU64 * ((blockIdx.x + blockIdx.y * 7u) % kWorkSlots);
      if (sa) atomicAdd(&slot[F32 ? 2 : 0], static_cast<unsigned long long>(sa));
      if (sb) atomicAdd(&slot[F32 ? 3 : 1], static_cast<unsigned long long>(sb));
    }
  }
}

// ---------------------------------------------------------------------------
// The vote kernel on staged records (ia_find_helices).  The same tiles,
// slices, lower bounds and outputs as k_vote, for events whose records fit
// (ev->rec_ok); the class-2 pairs of each evaluated triple are its records
// from k_stage, copied to LDS a chunk at a time, and the triple's frame
// comes from its TriFrame, so the kernel holds only the per-box arithmetic.
template <int BX, bool F32, bool EXACT = false>
__global__ void __launch_bounds__(kWG, 4) k_vote_rec(EvView vw, const BoxD* __restrict__ parents_all, Shape sh,
                                                  uint16_t* __restrict__ votes_all, uint32_t* __restrict__ hist_all,
                                                  uint32_t* __restrict__ status, const EventState* __restrict__ ev,
                                                  const int32_t* __restrict__ tlb_all,
                                                  const int32_t* __restrict__ tn2_all,
                                                  const int32_t* __restrict__ live_all,
                                                  const int32_t* __restrict__ live_off, int32_t n_ev,
                                                  const int32_t* __restrict__ rec_off_all, const void* __restrict__ rec,
                                                  const TriFrame* __restrict__ tfr_all,
                                                  int32_t* __restrict__ wg_max_all,
                                                  unsigned long long* __restrict__ work) {
  constexpr int HS = kWG / BX;
  constexpr int NQ = F32 ? 8 : 17;               // doubles of LDS per staged record
  static_assert(BX % 64 == 0 && HS * BX == kWG, "slices are whole waves");
  const uint32_t n_items = static_cast<uint32_t>(live_off[n_ev]);
  __shared__ double sq[NQ][kCap + 16];
  float(*sq32)[kCap + 16] = reinterpret_cast<float(*)[kCap + 16]>(&sq[0][0]);
  __shared__ int8_t sflag[kCap + 16];
  __shared__ int8_t stlive[kWG];
  __shared__ uint32_t shist[kHistLdsRec];
  __shared__ int32_t sred[HS][BX];
  __shared__ int32_t sbuf[kWG / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t bl = tid % BX, sl = tid / BX;
  auto triple_of = [&](uint32_t x) { return (x / sh.nc) * sh.m012 + (x % sh.nc) / sh.m34; };
  int32_t n_eval = 0;

  for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    // the item's event: the last one whose first item is at or before it
    int32_t elo = 0, ehi = n_ev - 1;
    while (elo < ehi) {
      const int32_t mid = (elo + ehi + 1) >> 1;
      if (static_cast<uint32_t>(live_off[mid]) <= item) elo = mid;
      else ehi = mid - 1;
    }
    const int e = elo;
    const int32_t n_hits = vw.count(e), n_bins = n_hits + 1;
    const BoxD* parents = parents_all + e * vw.par_stride;
    uint16_t* votes = votes_all + int64_t(e) * sh.n_boxes;
    uint32_t* hist = hist_all ? hist_all + int64_t(e) * vw.hist_stride : nullptr;
    const int32_t* tlb = tlb_all + e * vw.tri_stride;
    const int32_t* tn2 = tn2_all + e * vw.tri_stride;
    const int32_t* rec_off = rec_off_all + e * vw.tri_stride;
    const TriFrame* tfr = tfr_all + e * vw.tri_stride;
    int32_t* wg_max = wg_max_all + int64_t(e) * vw.wg_stride;
    const RecD* recd = reinterpret_cast<const RecD*>(rec) + int64_t(e) * vw.rec_stride;
    const PairQ32* recf = reinterpret_cast<const PairQ32*>(rec) + int64_t(e) * vw.rec_stride;
    const int32_t T = ev[e].t_prune;
    const int32_t tcut = ev[e].t_cut;
    const uint32_t tile = static_cast<uint32_t>(live_all[int64_t(e) * vw.wg_stride + (item - live_off[e])]);
    const uint32_t b0 = tile * BX;
    const uint32_t b_last = min(b0 + BX, sh.n_boxes) - 1;
    const uint32_t b = b0 + bl;
    const bool live = b < sh.n_boxes;
    const uint32_t bb = live ? b : b_last;
    const uint32_t t_first = triple_of(b0);
    const int32_t nt = static_cast<int32_t>(triple_of(b_last) - t_first + 1);
    const int32_t my_tl = static_cast<int32_t>(triple_of(bb) - t_first);
    const int32_t hc = max(1, kCap / nt);          // records per triple per chunk
    const int32_t pitch = hc + ((nt > 1 && nt <= 16) ? 1 : 0);

    __syncthreads();                     // LDS of the previous tile is free
    int32_t n2max = 0;
    for (int32_t i = tid; i < nt; i += kWG) {
      const int32_t a = tlb[t_first + i], c = tn2[t_first + i];
      const bool lv = c > 0 && triple_live(a, c, T, t_first + i, tcut);
      stlive[i] = lv ? 1 : 0;
      if (lv) n2max = max(n2max, c);
    }
    for (int o = 32; o > 0; o >>= 1) n2max = max(n2max, __shfl_down(n2max, o, 64));
    if ((tid & 63) == 0) sbuf[tid >> 6] = n2max;
    __syncthreads();
    n2max = 0;
    for (int w = 0; w < kWG / 64; ++w) n2max = max(n2max, sbuf[w]);

    const uint32_t my_t = t_first + my_tl;
    int32_t nv = sl == 0 ? tlb[my_t] : 0;
    if (n2max > 0) {                     // uniform over the workgroup (barriers below)
      const TriFrame fr = tfr[my_t];
      const Iv K = {fr.Klo, fr.Khi};
      uint32_t k[5];
      child_index(sh.m, bb % sh.nc, k);
      const BoxD& P = parents[bb / sh.nc];
      double zlo, zhi, llo, lhi;
      child_edge(P.lo[3], P.hi[3], sh.m[3], k[3], &zlo, &zhi);
      child_edge(P.lo[4], P.hi[4], sh.m[4], k[4], &llo, &lhi);
      const double z0 = 0.5 * (zlo + zhi), lam = 0.5 * (llo + lhi);
      const double lamR = lam * fr.R, lam2 = lam * lam;
      const float R32 = static_cast<float>(fr.R), sig32 = static_cast<float>(fr.sig);
      const Iv32 K32 = to32(K);
      const float z032 = static_cast<float>(z0), lam32 = static_cast<float>(lam);
      const float lamR32 = lam32 * R32, lam232 = lam32 * lam32;
      const int32_t my_n2 = stlive[my_tl] ? tn2[my_t] : 0;

      for (int32_t j0 = 0; j0 < n2max; j0 += hc) {
        __syncthreads();
        // copy records j0 .. j0 + hc - 1 of every evaluated triple to LDS
        for (int32_t r = tid; r < nt * hc; r += kWG) {
          const int32_t tl = r / hc, jl = r % hc;
          const int32_t slot = tl * pitch + jl;
          const uint32_t t = t_first + tl;
          if (!stlive[tl] || j0 + jl >= tn2[t]) { sflag[slot] = 0; continue; }
          const int64_t ri = int64_t(rec_off[t]) + j0 + jl;
          sflag[slot] = 2;
          if constexpr (F32) {
            const PairQ32 q = recf[ri];
            sq32[0][slot] = q.Glo; sq32[1][slot] = q.Ghi; sq32[2][slot] = q.sArc; sq32[3][slot] = q.dphi;
            sq32[4][slot] = q.RAx; sq32[5][slot] = q.sinA; sq32[6][slot] = q.cosA; sq32[7][slot] = q.sAx;
            sq32[8][slot] = q.cAx; sq32[9][slot] = q.c2; sq32[10][slot] = q.s2; sq32[11][slot] = q.twoRAx2;
            sq32[12][slot] = q.RpRAx; sq32[13][slot] = q.tt; sq32[14][slot] = q.d; sq32[15][slot] = q.bs;
          } else {
            const RecD& q = recd[ri];
            for (int c = 0; c < 12; ++c) sq[c][slot] = q.q[c];
            sq[12][slot] = recip_v(q.q[4]);     // RAx
            sq[13][slot] = drift_ok(q.d) ? recip_v(q.q[11]) : __builtin_nan("");   // twoRAx2, as pair_quantities
            sq[14][slot] = q.tt; sq[15][slot] = q.d; sq[16][slot] = q.band;
          }
        }
        __syncthreads();
        const int32_t nj = min(hc, my_n2 - j0);
        for (int32_t jl = sl; jl < nj; jl += HS) {
          const int32_t slot = my_tl * pitch + jl;
          n_eval += live ? 1 : 0;
          if constexpr (F32) {
            PairQ32 r;
            r.Glo = sq32[0][slot]; r.Ghi = sq32[1][slot]; r.sArc = sq32[2][slot]; r.dphi = sq32[3][slot];
            r.RAx = sq32[4][slot]; r.sinA = sq32[5][slot]; r.cosA = sq32[6][slot]; r.sAx = sq32[7][slot];
            r.cAx = sq32[8][slot]; r.c2 = sq32[9][slot]; r.s2 = sq32[10][slot]; r.twoRAx2 = sq32[11][slot];
            r.RpRAx = sq32[12][slot]; r.tt = sq32[13][slot]; r.d = sq32[14][slot]; r.bs = sq32[15][slot];
            if (stereo_vote32(r, R32, sig32, K32, z032, lam32, lamR32, lam232)) ++nv;
          } else {
            PairQ q;
            q.Glo = sq[0][slot]; q.Ghi = sq[1][slot]; q.sArc = sq[2][slot]; q.dphi = sq[3][slot];
            q.RAx = sq[4][slot]; q.sinA = sq[5][slot]; q.cosA = sq[6][slot]; q.sAx = sq[7][slot];
            q.cAx = sq[8][slot]; q.c2 = sq[9][slot]; q.s2 = sq[10][slot]; q.twoRAx2 = sq[11][slot];
            q.rRAx = sq[12][slot]; q.r2RAx2 = sq[13][slot];
            q.RpRAx = fr.R + q.RAx;            // as k_stage's pair_quantities forms it
            const double tt = sq[14][slot];
            if (stereo_vote<EXACT>(q, fr.R, fr.sig, K, z0, lam, lamR, lam2, tt, tt * tt, sq[15][slot], sq[16][slot]))
              ++nv;
          }
        }
      }
    }
    if (HS > 1) {
      __syncthreads();
      sred[sl][bl] = nv;
      __syncthreads();
      if (sl == 0)
        for (int s2 = 1; s2 < HS; ++s2) nv += sred[s2][bl];
    }
    const bool owner = sl == 0 && live;
    if (owner) votes[b] = static_cast<uint16_t>(nv);
    int32_t mv = owner ? nv : -1;
    for (int o = 32; o > 0; o >>= 1) mv = max(mv, __shfl_down(mv, o, 64));
    __syncthreads();
    if ((tid & 63) == 0) sbuf[tid >> 6] = mv;
    __syncthreads();
    int32_t wmax = -1;
    for (int w = 0; w < kWG / 64; ++w) wmax = max(wmax, sbuf[w]);
    if (tid == 0) wg_max[tile] = wmax;
    if (hist && wmax >= T) {
      const bool in_lds = n_bins <= kHistLdsRec;
      if (in_lds) {
        for (int32_t i = tid; i < n_bins; i += kWG) shist[i] = 0u;
        __syncthreads();
      }
      if (owner && nv >= T) {
        if (nv >= n_bins) atomicOr(status, kStVoteOverflow);
        else if (in_lds) atomicAdd(&shist[nv], 1u);
        else atomicAdd(&hist[nv], 1u);
      }
      if (in_lds) {
        __syncthreads();
        for (int32_t i = tid; i < n_bins; i += kWG)
          if (shist[i]) atomicAdd(&hist[i], shist[i]);
      }
    }
  }
  if (work) {
    int32_t a = n_eval;
    for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
    __syncthreads();
    if ((tid & 63) == 0) sbuf[tid >> 6] = a;
    __syncthreads();
    if (tid == 0) {
      int32_t sa = 0;
      for (int w = 0; w < kWG / 64; ++w) sa += sbuf[w];
      unsigned long long* slot = work + kWorkSlotU64 * (blockIdx.x % kWorkSlots);
      if (sa) atomicAdd(&slot[F32 ? 2 : 0], static_cast<unsigned long long>(sa));
    }
  }
}

// Offsets of each event's work items in one list over the batch, so that
// the workgroups of k_stage and of the vote kernel share the batch's items
// evenly: live_off[e] counts the live vote tiles of the events before e,
// stage_off[e] their (live triple, hit) pairs, and entry n_ev the totals.
// Events that are done, or whose records did not fit, count none.  One
// workgroup.
__global__ void __launch_bounds__(kWG) k_live_offsets(const EventState* __restrict__ ev, EvView vw, int32_t n_ev,
                                                      int32_t* __restrict__ live_off,
                                                      int64_t* __restrict__ stage_off) {
  __shared__ int32_t sbuf[kWG / 64];
  __shared__ int64_t s64[kWG];
  const int32_t per = (n_ev + kWG - 1) / kWG;
  const int32_t a = min(static_cast<int32_t>(threadIdx.x) * per, n_ev), b = min(a + per, n_ev);
  auto skip = [&](int32_t e) { return ev[e].done || !ev[e].rec_ok; };
  auto tiles = [&](int32_t e) { return skip(e) ? 0 : ev[e].n_live; };
  auto pairs = [&](int32_t e) {
    return skip(e) ? int64_t(0) : static_cast<int64_t>(ev[e].n_live_tri) * max(vw.count(e), 0);
  };
  int32_t c = 0;
  int64_t c2 = 0;
  for (int32_t e = a; e < b; ++e) { c += tiles(e); c2 += pairs(e); }
  int32_t pos;
  const int32_t total = block_scan_count(c, &pos, sbuf);
  // 64-bit exclusive scan of the pair counts (serial over the kWG partials)
  s64[threadIdx.x] = c2;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int w = 0; w < kWG; ++w) { const int64_t x = s64[w]; s64[w] = run; run += x; }
    stage_off[n_ev] = run;
  }
  __syncthreads();
  int64_t pos2 = s64[threadIdx.x];
  for (int32_t e = a; e < b; ++e) {
    live_off[e] = pos;
    pos += tiles(e);
    stage_off[e] = pos2;
    pos2 += pairs(e);
  }
  if (threadIdx.x == 0) live_off[n_ev] = total;
}

// ---------------------------------------------------------------------------
// histogram of an existing vote array (used when votes come from the caller)
__global__ void __launch_bounds__(kWG) k_hist(const uint16_t* __restrict__ votes, uint32_t n,
                                              uint32_t* __restrict__ hist, int32_t n_bins,
                                              uint32_t* __restrict__ status) {
  __shared__ uint32_t shist[kHistLds];
  const bool in_lds = n_bins <= kHistLds;
  if (in_lds) {
    for (int32_t i = threadIdx.x; i < n_bins; i += kWG) shist[i] = 0u;
    __syncthreads();
  }
  for (uint32_t i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    const int32_t v = votes[i];
    if (v >= n_bins) atomicOr(status, kStVoteOverflow);
    else if (in_lds) atomicAdd(&shist[v], 1u);
    else atomicAdd(&hist[v], 1u);
  }
  if (in_lds) {
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n_bins; i += kWG)
      if (shist[i]) atomicAdd(&hist[i], shist[i]);
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void __launch_bounds__(kWG) k_select_count(const uint16_t* __restrict__ votes, uint32_t n_boxes,
                                                      uint32_t chunk, const uint32_t* __restrict__ hist,
                                                      int32_t n_bins, int32_t k, int32_t* __restrict__ cnt,
                                                      const EventState* __restrict__ ev) {
  if (ev && ev->done) return;
  __shared__ SelInfo si;
  __shared__ int32_t sbuf[kWG / 64];
  if (threadIdx.x == 0) si = threshold(hist, n_bins, k, n_boxes);
  __syncthreads();
  const uint32_t beg = blockIdx.x * chunk, end = min(beg + chunk, n_boxes);
  int32_t gt = 0, eq = 0;
  for (uint32_t i = beg + threadIdx.x; i < end; i += kWG) {
    const int32_t v = votes[i];
    gt += v > si.vstar;
    eq += v == si.vstar;
  }
  gt = block_sum(gt, sbuf);
  eq = block_sum(eq, sbuf);
  if (threadIdx.x == 0) { cnt[2 * blockIdx.x] = gt; cnt[2 * blockIdx.x + 1] = eq; }
}

// writes the selection; the last workgroup to finish orders it, writes the
// selected boxes, clears the histogram and resets the completion counter.
__global__ void __launch_bounds__(kWG) k_select_write(
    const uint16_t* __restrict__ votes, uint32_t n_boxes, uint32_t chunk, uint32_t* __restrict__ hist,
    int32_t n_bins, int32_t k, const int32_t* __restrict__ cnt, uint32_t* __restrict__ tmp_idx,
    uint32_t* __restrict__ done_counter, const BoxD* __restrict__ parents, Shape sh,
    BoxD* __restrict__ out_boxes, int64_t* __restrict__ out_index, uint16_t* __restrict__ out_votes,
    EventState* __restrict__ ev, int32_t v_min_stop) {
  if (ev && ev->done) return;
  __shared__ SelInfo si;
  __shared__ int32_t sbuf[kWG / 64];
  __shared__ int32_t base_gt, base_eq;
  __shared__ int32_t is_last;
  __shared__ uint32_t s_idx[kMaxTopK];
  __shared__ uint16_t s_v[kMaxTopK];
  if (threadIdx.x == 0) si = threshold(hist, n_bins, k, n_boxes);
  __syncthreads();
  // prefix over earlier chunks
  int32_t pg = 0, pe = 0;
  for (int32_t w = threadIdx.x; w < static_cast<int32_t>(blockIdx.x); w += kWG) {
    pg += cnt[2 * w];
    pe += cnt[2 * w + 1];
  }
  pg = block_sum(pg, sbuf);
  pe = block_sum(pe, sbuf);
  if (threadIdx.x == 0) { base_gt = pg; base_eq = pe; }
  __syncthreads();
  const int32_t my_gt = cnt[2 * blockIdx.x], my_eq = cnt[2 * blockIdx.x + 1];
  const bool need = (my_gt > 0) || (my_eq > 0 && base_eq < si.need_eq);
  const uint32_t beg = blockIdx.x * chunk, end = min(beg + chunk, n_boxes);
  int32_t run_gt = base_gt, run_eq = base_eq;
  const int32_t stop_gt = base_gt + my_gt;
  const int32_t stop_eq = min(base_eq + my_eq, si.need_eq);
  for (uint32_t i0 = beg; need && i0 < end && (run_gt < stop_gt || run_eq < stop_eq); i0 += kWG) {
    const uint32_t i = i0 + threadIdx.x;
    const int32_t v = i < end ? votes[i] : -1;
    const int32_t fg = v > si.vstar, fe = v == si.vstar;
    int32_t xg, xe;
    const int32_t tg = block_scan(fg, &xg, sbuf);
    const int32_t te = block_scan(fe, &xe, sbuf);
    if (fg && run_gt + xg < si.n_gt) tmp_idx[run_gt + xg] = i;
    if (fe && run_eq + xe < si.need_eq) tmp_idx[si.n_gt + run_eq + xe] = i;
    run_gt += tg;
    run_eq += te;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(done_counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  __shared__ int32_t s_vmax;
  __shared__ uint32_t s_nmax;
  if (threadIdx.x == 0) {
    int32_t vm = 0;
    uint32_t nm = 0;
    for (int32_t v = n_bins - 1; v >= 0; --v) {
      const uint32_t c = hist[v];
      if (c != 0u) { vm = v; nm = c; break; }
    }
    s_vmax = vm;
    s_nmax = nm;
  }
  const int32_t ke = si.k_eff;
  for (int32_t a = threadIdx.x; a < ke; a += kWG) {
    const uint32_t ia = __atomic_load_n(&tmp_idx[a], __ATOMIC_RELAXED);
    s_idx[a] = ia;
    s_v[a] = votes[ia];
  }
  __syncthreads();
  // order the k_eff entries by (votes desc, index asc)
  for (int32_t a = threadIdx.x; a < ke; a += kWG) {
    const uint32_t ia = s_idx[a];
    const int32_t va = s_v[a];
    int32_t rank = 0;
    for (int32_t c = 0; c < ke; ++c) {
      const int32_t vc = s_v[c];
      rank += (vc > va) || (vc == va && s_idx[c] < ia);
    }
    out_index[rank] = ia;
    out_votes[rank] = static_cast<uint16_t>(va);
    if (out_boxes) level_box(parents, sh, ia, &out_boxes[rank]);
  }
  __syncthreads();
  for (int32_t i = threadIdx.x; i < n_bins; i += kWG) hist[i] = 0u;
  if (threadIdx.x == 0) {
    *done_counter = 0u;
    if (ev) {
      ev->vmax = s_vmax;
      ev->n_argmax = static_cast<int32_t>(s_nmax);
      ev->k_sel = ke;
      if (v_min_stop > 0 && s_vmax < v_min_stop) ev->done = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// estimate from the max-vote cells of a level (Sec. 3.3): mean of the cell
// centres (phi0 relative to the first cell's centre, in (-pi, pi]) and half
// the extent of their union.  Sums are pairwise over the level's boxes in
// index order on a zero-padded power-of-two array: k_est_partial reduces
// aligned 256-box chunks (one box per lane, adjacent pairs in LDS; a
// workgroup takes `per` consecutive chunks in turn, at most kEstPer, fewer
// for small launches), and k_est_final reduces the chunk sums on the same
// tree.  vmax and the first
// max-vote box come from the level's selection (rank 0).
struct EstimateOut {
  double p[5], err[5];
  int32_t vmax, n_argmax;
};

constexpr int kEstQ = 16;        // 5 sums, 5 minima, 5 maxima, count
constexpr int kEstPer = 16;      // chunks per k_est_partial workgroup
static_assert(kEstPer <= 32, "chunks_reaching keeps one bit per chunk of a workgroup");

// Which of a workgroup's 256-box chunks [c0, c1) (at most 32) can hold a
// box with `vlo` votes or more: bit ch - c0 is clear when the chunk lies past
// the level's boxes or every vote tile it overlaps (tiles of bx boxes, bx =
// 64, 128 or 256) has its maximum below vlo.  The tile maxima are read once,
// spread over the workgroup's threads, so the chunks' own loop needs no
// further global read to skip a chunk.  Call from every thread; the result
// is the same for all.
__device__ uint32_t chunks_reaching(const int32_t* wg_max, int32_t bx, uint32_t c0, uint32_t c1, uint32_t n_boxes,
                                    int32_t vlo, uint32_t* smask) {
  const uint32_t b0 = c0 * static_cast<uint32_t>(kWG);
  if (threadIdx.x == 0) *smask = 0u;
  __syncthreads();
  if (b0 < n_boxes) {
    const uint32_t b1 = min(c1 * static_cast<uint32_t>(kWG), n_boxes) - 1;
    if (!wg_max) {
      if (threadIdx.x == 0) *smask = (b1 / kWG - c0 == 31) ? 0xffffffffu : ((2u << (b1 / kWG - c0)) - 1u);
    } else {
      const uint32_t ub = static_cast<uint32_t>(bx);
      for (uint32_t t = b0 / ub + threadIdx.x; t <= b1 / ub; t += kWG)
        if (wg_max[t] >= vlo) atomicOr(smask, 1u << ((t * ub) / kWG - c0));
    }
  }
  __syncthreads();
  return *smask;
}

__device__ __forceinline__ void tree_step(double (*s)[kWG], int w) {
  // s[q][i] = combine(s[q][2i], s[q][2i + 1]) for i < w / 2
  const int t = threadIdx.x;
  double v[kEstQ];
  const bool act = t < w / 2;
  if (act) {
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] = s[q][2 * t] + s[q][2 * t + 1];
#pragma unroll
    for (int q = 5; q < 10; ++q) v[q] = fmin(s[q][2 * t], s[q][2 * t + 1]);
#pragma unroll
    for (int q = 10; q < 15; ++q) v[q] = fmax(s[q][2 * t], s[q][2 * t + 1]);
    v[15] = s[15][2 * t] + s[15][2 * t + 1];
  }
  __syncthreads();
  if (act)
#pragma unroll
    for (int q = 0; q < kEstQ; ++q) s[q][t] = v[q];
  __syncthreads();
}

__global__ void __launch_bounds__(kWG) k_est_partial(const BoxD* __restrict__ parents, Shape sh,
                                                     const uint16_t* __restrict__ votes,
                                                     const BoxD* __restrict__ first_box,
                                                     const uint16_t* __restrict__ first_votes,
                                                     double* __restrict__ part, EvView vw,
                                                     const EventState* __restrict__ ev,
                                                     const int32_t* __restrict__ wg_max, int32_t bx,
                                                     uint32_t n_part, uint32_t per, int32_t use_run,
                                                     const int32_t* __restrict__ live_list,
                                                     uint32_t* __restrict__ emask, int32_t emask_stride) {
  const int e = blockIdx.y;
  if (ev && ev[e].done) return;
  parents += e * vw.par_stride;
  votes += int64_t(e) * sh.n_boxes;
  if (wg_max) wg_max += int64_t(e) * vw.wg_stride;
  first_box += int64_t(e) * vw.k;
  first_votes += int64_t(e) * vw.k;
  part += int64_t(e) * vw.part_stride;
  __shared__ double s[kEstQ][kWG];
  const int32_t vmax = first_votes[0];
  const double c0 = 0.5 * (first_box->lo[1] + first_box->hi[1]);
  const int32_t ra = use_run ? ev[e].run_a : -1, rb = use_run ? ev[e].run_b : -1;
  // one chunk: its record on the pairwise tree of its 256 lanes; a chunk
  // without a max-vote box reduces to the identity (sums 0, minima +inf,
  // maxima -inf, count 0), bit for bit, written without the tree (dense) or
  // left to k_est_final as a clear bit of emask (sparse)
  auto chunk = [&](uint32_t ch, bool may) {
    const uint32_t i = ch * kWG + threadIdx.x;
    double v[kEstQ];
    for (int q = 0; q < 5; ++q) { v[q] = 0.0; v[5 + q] = INFINITY; v[10 + q] = -INFINITY; }
    v[15] = 0.0;
    // with wg_max, only tiles whose maximum reaches vmax hold written votes
    const bool at_max = may && i < sh.n_boxes && (!wg_max || wg_max[i / static_cast<uint32_t>(bx)] >= vmax) &&
                        votes[i] == vmax && in_run(phi_bin(sh, i), ra, rb);
    if (!may || !__syncthreads_or(at_max ? 1 : 0)) {
      if (!emask && threadIdx.x < kEstQ) {
        const int q = static_cast<int>(threadIdx.x);
        part[ch * kEstQ + q] = (q >= 5 && q < 10) ? INFINITY : ((q >= 10 && q < 15) ? -INFINITY : 0.0);
      }
      return;
    }
    if (at_max) {
      BoxD box;
      level_box(parents, sh, i, &box);
      for (int j = 0; j < 5; ++j) {
        double lo = box.lo[j], hi = box.hi[j];
        const double c = 0.5 * (lo + hi);
        if (j == 1) {
          const double dv = c - c0;
          double shift = 0.0;
          if (dv > kPi) shift = -kTwoPi;
          else if (dv <= -kPi) shift = kTwoPi;
          v[j] = dv + shift;
          lo = lo + shift;
          hi = hi + shift;
        } else {
          v[j] = c;
        }
        v[5 + j] = lo;
        v[10 + j] = hi;
      }
      v[15] = 1.0;
    }
    for (int q = 0; q < kEstQ; ++q) s[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kWG; w > 1; w >>= 1) tree_step(s, w);
    if (threadIdx.x < kEstQ) part[ch * kEstQ + threadIdx.x] = s[threadIdx.x][0];
    if (emask && threadIdx.x == 0) atomicOr(&emask[ch >> 5], 1u << (ch & 31u));
    __syncthreads();                           // s is refilled for the next chunk
  };
  if (emask) {
    // sparse: only chunks holding a live tile (every box with written votes
    // lies in one), each taken by the workgroup of its first live tile
    emask += int64_t(e) * emask_stride;
    live_list += int64_t(e) * vw.wg_stride;
    const int32_t n_live = ev[e].n_live;
    const uint32_t ub = static_cast<uint32_t>(bx), per_ch = static_cast<uint32_t>(kWG) / ub;
    for (int32_t li = blockIdx.x; li < n_live; li += gridDim.x) {
      const uint32_t ch = static_cast<uint32_t>(live_list[li]) / per_ch;
      if (li > 0 && static_cast<uint32_t>(live_list[li - 1]) / per_ch == ch) continue;
      int32_t mx = -1;
      for (uint32_t t = ch * per_ch; t < min((ch + 1) * per_ch, (sh.n_boxes + ub - 1) / ub); ++t)
        mx = max(mx, wg_max[t]);
      chunk(ch, mx >= vmax);
    }
    return;
  }
  const uint32_t ch_end = min(n_part, (blockIdx.x + 1) * per);
  __shared__ uint32_t smask;
  const uint32_t reach = chunks_reaching(wg_max, bx, blockIdx.x * per, ch_end, sh.n_boxes, vmax, &smask);
  for (uint32_t ch = blockIdx.x * per; ch < ch_end; ++ch) chunk(ch, (reach >> (ch - blockIdx.x * per)) & 1u);
}

// hit finding (Sec. 3.3): does an active hit vote for the box estimate +- scale x error
IA_HD bool pair_vote_box(const BoxD& b, const HitRec& h, bool fwd = false, bool exact = false) {
  if (!h.use) return false;
  Frame f;
  f.Dd = {b.lo[0], b.hi[0]};
  f.Fi = {b.lo[1], b.hi[1]};
  f.K = {b.lo[2], b.hi[2]};
  if (fwd && !forward_ok(f.Fi, h)) return false;
  double c0 = 0.5 * (f.Dd.lo + f.Dd.hi), c1 = 0.5 * (f.Fi.lo + f.Fi.hi), kap = 0.5 * (f.K.lo + f.K.hi);
  double sig = 1.0;
  if (kap < 0.0) sig = -1.0;
  if (kap == 0.0) { kap = 0x1p-30; sig = 1.0; }
  const double kp = sig * kap, d0p = sig * c0;
  f.sp0 = sig * sin_p(c1);
  f.cp0 = cos_p(c1);
  f.R = 1.0 / kp;
  const double Rd = f.R + d0p;
  f.xc = -(Rd * f.sp0);
  f.yc = Rd * f.cp0;
  f.sig = sig;
  const Iv G = residual_G(f, h);
  if (h.axial)
    return h_contains0(G, f.K, f.sig * h.d, h.band) || h_contains0(G, f.K, f.sig * (-h.d), h.band);
  const PairQ q = pair_quantities(f, h, G);
  const double z0 = 0.5 * (b.lo[3] + b.hi[3]), lam = 0.5 * (b.lo[4] + b.hi[4]);
  if (exact)
    return stereo_vote<true>(q, f.R, f.sig, f.K, z0, lam, lam * f.R, lam * lam, h.tant, h.tant * h.tant, h.d, h.band);
  return stereo_vote(q, f.R, f.sig, f.K, z0, lam, lam * f.R, lam * lam, h.tant, h.tant * h.tant, h.d, h.band);
}

// helix record: {p[5], err[5], votes, n_assigned, n_argmax, status}
struct HelixOut {
  double p[5], err[5], ref[2];
  int32_t votes, n_assigned, n_argmax, status;
};

// One workgroup: combines the n_part chunk sums (n_part a power of two) on
// the pairwise tree, writes the estimate; with `hits` set it then runs hit
// finding for the event and records the helix.
// With `ev` set and `hits` null it only records the estimate and the union of
// the max-vote boxes in the event state (a level of the window schedule).
// Hit finding applies the forward-hit test when fwd is set, in the level's
// frame; the helix's p is taken back to the origin.
__global__ void __launch_bounds__(kWG) k_est_final(const double* __restrict__ part, int32_t n_part,
                                                   const BoxD* __restrict__ first_box,
                                                   const uint16_t* __restrict__ first_votes,
                                                   EstimateOut* __restrict__ out, EventState* __restrict__ ev,
                                                   HitRec* __restrict__ hits, EvView vw, double scale,
                                                   int32_t* __restrict__ assigned, HelixOut* __restrict__ hout,
                                                   int32_t* __restrict__ n_out, int32_t fwd,
                                                   uint32_t* __restrict__ emask, int32_t emask_stride) {
  const int e = blockIdx.y;
  if (ev && ev[e].done) return;
  part += int64_t(e) * vw.part_stride;
  if (emask) emask += int64_t(e) * emask_stride;
  // with emask, a chunk whose bit is clear holds the identity (k_est_partial
  // wrote no record for it): the same values enter the tree, unread
  auto has = [&](int32_t i) { return !emask || ((emask[i >> 5] >> (i & 31)) & 1u); };
  first_box += int64_t(e) * vw.k;
  first_votes += int64_t(e) * vw.k;
  if (ev) ev += e;
  const int32_t n_hits = vw.count(e), max_out = vw.max_out;
  if (hits) hits += vw.beg(e);
  if (assigned) assigned += vw.beg(e);
  if (hout) hout += int64_t(e) * max_out;
  if (n_out) n_out += e;
  __shared__ double s[kEstQ][kWG];
  __shared__ double stack[kWG][kEstLevels];
  __shared__ double sp[5], se[5];
  __shared__ int32_t s_count, s_assigned;
  const int t = threadIdx.x;
  // each lane reduces `seg` consecutive chunk sums with a binary-counter stack
  const int32_t nthr = min(kWG, n_part);
  const int32_t seg = n_part / nthr;
  for (int q = 0; q < kEstQ; ++q) {
    double acc = 0.0;
    if (t < nthr) {
      const int32_t beg = t * seg;
      if (q < 5 || q == 15) {
        for (int32_t i = 0; i < seg; ++i) {
          double v = has(beg + i) ? part[(beg + i) * kEstQ + q] : 0.0;
          int32_t c = i, lvl = 0;
          while (c & 1) { v = stack[t][lvl] + v; c >>= 1; ++lvl; }
          stack[t][lvl] = v;
        }
        int lg = 0;
        while ((1 << lg) < seg) ++lg;
        acc = stack[t][lg];
      } else {
        acc = q < 10 ? INFINITY : -INFINITY;
        for (int32_t i = 0; i < seg; ++i) {
          if (!has(beg + i)) continue;         // fmin(acc, +inf) = acc, fmax(acc, -inf) = acc
          const double v = part[(beg + i) * kEstQ + q];
          acc = q < 10 ? fmin(acc, v) : fmax(acc, v);
        }
      }
    } else {
      acc = (q >= 5 && q < 10) ? INFINITY : ((q >= 10 && q < 15) ? -INFINITY : 0.0);
    }
    s[q][t] = acc;
  }
  __syncthreads();
  if (emask)                                   // cleared for the next level
    for (int32_t w = t; w < (n_part + 31) / 32; w += kWG) emask[w] = 0u;
  for (int w = kWG; w > 1; w >>= 1) tree_step(s, w);
  if (t == 0) {
    const double c0 = 0.5 * (first_box->lo[1] + first_box->hi[1]);
    const int32_t count = static_cast<int32_t>(s[15][0]);
    for (int j = 0; j < 5; ++j) {
      const double S = s[j][0];
      double pj;
      if (j == 1) {
        pj = c0 + S / static_cast<double>(count);
        if (pj < 0.0) pj += kTwoPi;
        if (pj >= kTwoPi) pj -= kTwoPi;
      } else {
        pj = S / static_cast<double>(count);
      }
      sp[j] = pj;
      se[j] = 0.5 * (s[10 + j][0] - s[5 + j][0]);
    }
    s_count = count;
    s_assigned = 0;
    if (out) {
      for (int j = 0; j < 5; ++j) { out->p[j] = sp[j]; out->err[j] = se[j]; }
      out->vmax = first_votes[0];
      out->n_argmax = count;
    }
    if (ev && !hits) {
      for (int j = 0; j < 5; ++j) {
        ev->p[j] = sp[j];
        ev->err[j] = se[j];
        ev->ulo[j] = s[5 + j][0];
        ev->uhi[j] = s[10 + j][0];
      }
      ev->n_argmax = count;
    }
  }
  __syncthreads();
  if (!ev || !hits) return;
  // hit finding: every still-active hit voting for estimate +- scale x error
  BoxD E;
  for (int j = 0; j < 5; ++j) {
    const double w = scale * se[j];
    E.lo[j] = sp[j] - w;
    E.hi[j] = sp[j] + w;
  }
  const int32_t k = ev->n_out;
  int32_t mine = 0;
  for (int32_t i = t; i < n_hits; i += kWG) {
    if (pair_vote_box(E, hits[i], (fwd & 1) && !ev->moved, (fwd & 2) != 0)) {
      hits[i].use = 0;
      if (assigned) assigned[i] = k;
      ++mine;
    }
  }
  if (mine) atomicAdd(&s_assigned, mine);
  __syncthreads();
  if (t == 0) {
    const int32_t na = s_assigned;
    if (k < max_out) {
      HelixOut h;
      double p0[5] = {sp[0], sp[1], sp[2], sp[3], sp[4]};
      if (ev->moved) frame_shift(sp, -ev->ref[0], -ev->ref[1], p0);
      for (int j = 0; j < 5; ++j) { h.p[j] = p0[j]; h.err[j] = se[j]; }
      h.ref[0] = ev->ref[0];
      h.ref[1] = ev->ref[1];
      h.votes = first_votes[0];
      h.n_assigned = na;
      h.n_argmax = s_count;
      h.status = 0;
      hout[k] = h;
      ev->n_out = k + 1;
    }
    for (int j = 0; j < 5; ++j) { ev->p[j] = sp[j]; ev->err[j] = se[j]; }
    ev->n_assigned = na;
    ev->n_argmax = s_count;
    if (n_out) *n_out = ev->n_out;
    if (na == 0 || ev->n_out >= max_out) ev->done = 1;
  }
}

// ---------------------------------------------------------------------------
// IV levels: d^Ax enclosed over the whole box instead of its value at the
// middle of the voxel (Sec. 3.1), every quantity of Appendix A in interval
// arithmetic in the box's kappa > 0 frame, Phi - Phi^Ax enclosed by interval
// fixed-point steps of Eq. CSAXtoPHI_a from [-pi, pi] (each step keeps every
// solution); the same operations in the same order as the oracle's.
constexpr int kIvIters = 6;

struct IvSt { Iv sinP, cosP, u, delta, zS, ld, ctau; };

IA_HD bool iv_stereo_point(Iv EPS, Iv SINA, Iv COSA, Iv LAM, double tt, Iv T2, double dS, Iv R, Iv DPHI, Iv Z0,
                           Iv CAX, Iv SAX, IvSt* o) {
  const Iv SE = sin_encl(EPS.lo, EPS.hi), CE = cos_encl(EPS.lo, EPS.hi);
  o->sinP = iadd(imul(SINA, CE), imul(COSA, SE));
  o->cosP = isub(imul(COSA, CE), imul(SINA, SE));
  const Iv U2 = iadd(iadd(iadd(ipt(1.0), imul_pt(imul(itwice(LAM), o->sinP), tt)), imul(isqr(LAM), T2)),
                     imul(isqr(o->cosP), T2));
  if (!(U2.lo > 0.0)) return false;
  o->u = isqrt(U2);
  o->delta = idiv_pos(ipt(dS), o->u);
  const Iv SPERP = imul(R, iadd(DPHI, EPS));
  o->zS = isub(iadd(Z0, imul(LAM, SPERP)), imul_pt(imul(o->delta, o->cosP), tt));
  o->ld = imul(LAM, o->delta);
  o->ctau = isub(imul(o->zS, CAX), imul(o->ld, SAX));
  return true;
}

// enclosure of e = sgn(kappa) d^Ax over box b for drift sign s; false when
// none (kappa of both signs, a bound that fails): the pair then votes
IA_HD bool stereo_encl(const BoxD& b, const HitRec& h, int s, Iv* out) {
  if (b.lo[2] <= 0.0 && b.hi[2] >= 0.0) return false;
  const double sig = b.lo[2] > 0.0 ? 1.0 : -1.0;
  const Iv K = {b.lo[2], b.hi[2]}, D0 = {b.lo[0], b.hi[0]}, FI = {b.lo[1], b.hi[1]};
  const double dS = static_cast<double>(s) * h.d;
  if (h.axial) {
    *out = {sig * dS, sig * dS};
    return true;
  }
  const Iv KP = sig > 0.0 ? K : ineg(K), D0P = sig > 0.0 ? D0 : ineg(D0);
  const Iv SF = sin_encl(FI.lo, FI.hi), CP0 = cos_encl(FI.lo, FI.hi);
  const Iv SP0 = sig > 0.0 ? SF : ineg(SF);
  const Iv R = {wdn(1.0 / KP.hi), wup(1.0 / KP.lo)};
  const Iv RD = iadd(R, D0P);
  const Iv XC = ineg(imul(RD, SP0)), YC = imul(RD, CP0);
  const double py = sig * h.py, cps = sig * h.cphis, sps = h.sphis;
  const Iv DX = isub(ipt(h.px), XC), DY = isub(ipt(py), YC);
  const Iv RAX2 = iadd(isqr(DX), isqr(DY));
  if (!(RAX2.lo > 0.0)) return false;
  const Iv RAX = isqrt(RAX2);
  const Iv CAX = isub(imul_pt(DX, sps), imul_pt(DY, cps));
  const Iv SAX = iadd(imul_pt(DX, cps), imul_pt(DY, sps));
  const Iv SINA = idiv_pos(SAX, RAX), COSA = idiv_pos(CAX, RAX);
  const Iv YY = iadd(imul(DX, CP0), imul(DY, SP0)), XX = isub(imul(DX, SP0), imul(DY, CP0));
  const Iv DPHI = atan2_encl(YY, XX);
  const Iv Z0 = {b.lo[3], b.hi[3]}, LAM = {b.lo[4], b.hi[4]};
  const double tt = h.tant;
  const Iv T2 = {wdn(tt * tt), wup(tt * tt)};
  Iv EPS = {-2.0 * kPio2Up, 2.0 * kPio2Up};
  IvSt q;
  for (int k = 0; k < kIvIters; ++k) {
    if (!iv_stereo_point(EPS, SINA, COSA, LAM, tt, T2, dS, R, DPHI, Z0, CAX, SAX, &q)) return false;
    const Iv ST = ineg(iadd(imul(q.ld, CAX), imul(q.zS, SAX)));
    const Iv DEN = iadd(RAX2, imul_pt(q.ctau, tt));
    if (!(DEN.lo > 0.0)) return false;
    const Iv F = atan2_encl(imul_pt(ST, tt), DEN);
    EPS.lo = fmax(EPS.lo, F.lo);
    EPS.hi = fmin(EPS.hi, F.hi);
    if (!(EPS.lo <= EPS.hi)) return false;
  }
  if (!iv_stereo_point(EPS, SINA, COSA, LAM, tt, T2, dS, R, DPHI, Z0, CAX, SAX, &q)) return false;
  const Iv A1 = imul_pt(q.zS, tt), A2 = imul_pt(q.ld, tt);
  const Iv Q = iadd(iadd(imul_pt(itwice(q.ctau), tt), isqr(A1)), isqr(A2));
  const Iv A = iadd(R, q.delta);
  const Iv DISC = isub(isqr(A), Q);
  if (!(DISC.lo > 0.0) || !(A.lo > 0.0)) return false;
  const Iv DHAT = isub(q.delta, idiv_pos(Q, iadd(A, isqrt(DISC))));
  const Iv E = sig > 0.0 ? DHAT : ineg(DHAT);
  if (!__builtin_isfinite(E.lo) || !__builtin_isfinite(E.hi)) return false;
  *out = E;
  return true;
}

// the IV vote of a stereo (box, hit) pair: zero in 2G - 2E - kappa E^2 for
// either sign, E the box enclosure widened by the band
IA_HD bool pair_vote_iv(const BoxD& b, const HitRec& h, Iv G) {
  const Iv K = {b.lo[2], b.hi[2]};
  for (int si = 0; si < 2; ++si) {
    Iv E;
    if (!stereo_encl(b, h, si == 0 ? 1 : -1, &E)) return true;
    const Iv Eb = {wdn(E.lo - h.band), wup(E.hi + h.band)};
    const Iv Hb = isub(itwice(G), iadd(itwice(Eb), imul(K, isqr(Eb))));
    if (Hb.lo <= 0.0 && 0.0 <= Hb.hi) return true;
  }
  return false;
}

// The vote of an IV level: one lane per box (tiles of kWG boxes), over the
// batch's live tiles (live_all, offsets live_off) or, without a list, every
// tile of n_ev events; each box starts from its triple's lower bound and
// adds the class-2 stereo pairs it gets.  Outputs as k_vote_rec's.
__global__ void __launch_bounds__(kWG) k_vote_iv(const HitRec* __restrict__ hits_all, EvView vw,
                                                 const BoxD* __restrict__ parents_all, Shape sh,
                                                 const uint8_t* __restrict__ flags_all, uint16_t* __restrict__ votes_all,
                                                 uint32_t* __restrict__ hist_all, uint32_t* __restrict__ status,
                                                 const EventState* __restrict__ ev, const int32_t* __restrict__ tlb_all,
                                                 const int32_t* __restrict__ tn2_all,
                                                 const int32_t* __restrict__ live_all,
                                                 const int32_t* __restrict__ live_off, int32_t n_ev,
                                                 int32_t* __restrict__ wg_max_all,
                                                 unsigned long long* __restrict__ work) {
  const uint32_t n_tr = sh.n_parents * sh.m012;
  const uint32_t n_tiles = (sh.n_boxes + kWG - 1) / kWG;
  const uint32_t n_items = live_all ? static_cast<uint32_t>(live_off[n_ev]) : n_tiles * static_cast<uint32_t>(n_ev);
  __shared__ uint32_t shist[kHistLds];
  __shared__ int32_t sbuf[kWG / 64];
  const uint32_t tid = threadIdx.x;
  auto triple_of = [&](uint32_t x) { return (x / sh.nc) * sh.m012 + (x % sh.nc) / sh.m34; };
  int32_t n_eval = 0;
  for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    int e;
    uint32_t tile;
    if (live_all) {
      int32_t elo = 0, ehi = n_ev - 1;
      while (elo < ehi) {
        const int32_t mid = (elo + ehi + 1) >> 1;
        if (static_cast<uint32_t>(live_off[mid]) <= item) elo = mid;
        else ehi = mid - 1;
      }
      e = elo;
      tile = static_cast<uint32_t>(live_all[int64_t(e) * vw.wg_stride + (item - live_off[e])]);
    } else {
      e = static_cast<int>(item / n_tiles);
      tile = item % n_tiles;
    }
    const int32_t n_hits = vw.count(e), n_bins = n_hits + 1;
    const HitRec* hits = hits_all + vw.beg(e);
    const BoxD* parents = parents_all + e * vw.par_stride;
    const uint8_t* flags = flags_all + e * vw.flag_stride;
    const int32_t* tlb = tlb_all + e * vw.tri_stride;
    const int32_t* tn2 = tn2_all + e * vw.tri_stride;
    uint16_t* votes = votes_all + int64_t(e) * sh.n_boxes;
    uint32_t* hist = hist_all ? hist_all + int64_t(e) * vw.hist_stride : nullptr;
    int32_t* wg_max = wg_max_all ? wg_max_all + int64_t(e) * vw.wg_stride : nullptr;
    const int32_t T = ev ? ev[e].t_prune : 0;
    const int32_t tcut = ev ? ev[e].t_cut : INT32_MAX;
    const uint32_t b = tile * kWG + tid;
    const bool live = b < sh.n_boxes;
    const uint32_t t = triple_of(live ? b : sh.n_boxes - 1);
    int32_t nv = tlb[t];
    if (live && tn2[t] > 0 && triple_live(tlb[t], tn2[t], T, t, tcut)) {
      const BoxD& P = parents[b / sh.nc];
      BoxD B;
      child_box(P, sh.m, b % sh.nc, &B);
      const uint32_t tc = t % sh.m012;
      const Frame f = triple_frame(P, sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
      for (int32_t h = 0; h < n_hits; ++h) {
        if (flags[int64_t(h) * n_tr + t] != 2) continue;
        const HitRec hr = hits[h];
        ++n_eval;
        if (pair_vote_iv(B, hr, residual_G(f, hr))) ++nv;
      }
    }
    if (live) votes[b] = static_cast<uint16_t>(nv);
    int32_t mv = live ? nv : -1;
    for (int o = 32; o > 0; o >>= 1) mv = max(mv, __shfl_down(mv, o, 64));
    __syncthreads();
    if ((tid & 63) == 0) sbuf[tid >> 6] = mv;
    __syncthreads();
    int32_t wmax = -1;
    for (int w = 0; w < kWG / 64; ++w) wmax = max(wmax, sbuf[w]);
    if (wg_max && tid == 0) wg_max[tile] = wmax;
    if (hist && wmax >= T) {
      const bool in_lds = n_bins <= kHistLds;
      if (in_lds) {
        for (int32_t i = tid; i < n_bins; i += kWG) shist[i] = 0u;
        __syncthreads();
      }
      if (live && nv >= T) {
        if (nv >= n_bins) atomicOr(status, kStVoteOverflow);
        else if (in_lds) atomicAdd(&shist[nv], 1u);
        else atomicAdd(&hist[nv], 1u);
      }
      if (in_lds) {
        __syncthreads();
        for (int32_t i = tid; i < n_bins; i += kWG)
          if (shist[i]) atomicAdd(&hist[i], shist[i]);
      }
    }
  }
  if (work) {
    int32_t a = n_eval;
    for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
    if ((tid & 63) == 0 && a) {
      unsigned long long* slot = work + kWorkSlotU64 * ((blockIdx.x * 4u + (tid >> 6)) % kWorkSlots);
      atomicAdd(&slot[0], static_cast<unsigned long long>(a));
    }
  }
}

// ---------------------------------------------------------------------------
// Resident pools (continuous batching): events sit in fixed-size rows of
// max_hits hits, row r starting at hit r * max_hits; a row holds the whole
// per-event search state between helix passes.

// an empty pool: every row done, no hits, the search range in place
__global__ void k_pool_init(int32_t* __restrict__ off, int32_t* __restrict__ cnt, EventState* __restrict__ ev,
                            int32_t* __restrict__ n_out, int32_t rows, int32_t max_hits,
                            BoxD* __restrict__ range_dst, BoxD range) {
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r <= rows; r += stride) {
    off[r] = r * max_hits;
    if (r == rows) continue;
    cnt[r] = 0;
    EventState es{};
    es.done = 1;
    es.t_cut = INT32_MAX;
    ev[r] = es;
    n_out[r] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *range_dst = range;
}

// copies new event j (hits new_off[j] .. new_off[j+1] of src) into row
// new_rows[j] of the pool's hit store; the host has checked the sizes
__global__ void k_pool_load(const double* __restrict__ src, const int32_t* __restrict__ new_off,
                            const int32_t* __restrict__ new_rows, double* __restrict__ store,
                            int32_t* __restrict__ cnt, int32_t max_hits) {
  const int32_t j = blockIdx.y;
  const int32_t r = new_rows[j], b = new_off[j], n = new_off[j + 1] - b;
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[r] = n;
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n * 8; i += stride)
    store[(int64_t(r) * max_hits) * 8 + i] = src[int64_t(b) * 8 + i];
}

// per row: done flag and helices written, for the host's poll
__global__ void k_pool_state(const EventState* __restrict__ ev, const int32_t* __restrict__ n_out, int32_t rows,
                             int32_t* __restrict__ dst) {
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += stride) {
    dst[2 * r] = ev[r].done;
    dst[2 * r + 1] = n_out[r];
  }
}

// ---------------------------------------------------------------------------
// Window schedule (Sec. 3.3, Table 1): every level is one grid over a window
// box per event.  The kernels below build the next window from all max-vote
// boxes of a level and move the reference point of the parametrisation.

// Re-prepares every hit of an event about its reference point, keeping each
// hit's use flag (reset: about the origin, the event's frame is reset and
// every active hit votes again).
__global__ void __launch_bounds__(kWG) k_reframe(const double* __restrict__ hits, EvView vw,
                                                 HitRec* __restrict__ out, EventState* __restrict__ ev,
                                                 int32_t reset) {
  const int e = blockIdx.y;
  if (ev[e].done) return;
  const int32_t beg = vw.beg(e), n_hits = vw.count(e);
  const double xr = reset ? 0.0 : ev[e].ref[0], yr = reset ? 0.0 : ev[e].ref[1];
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < n_hits; h += stride) {
    HitRec r;
    bool bad;
    const int32_t use = out[beg + h].use;
    prep_one(hits + 8 * static_cast<int64_t>(beg + h), use != 0, &r, &bad, xr, yr);
    r.use = reset ? (use & 1) : use;     // a pass starts with every active hit voting
    out[beg + h] = r;
  }
  if (reset && blockIdx.x == 0 && threadIdx.x == 0) {
    ev[e].ref[0] = 0.0;
    ev[e].ref[1] = 0.0;
    ev[e].moved = 0;
  }
}

// The measurement point closest to the recovered circle: the active hit with
// the smallest |G| at the estimate, the lowest index on ties.  One workgroup
// per event; sets `moving` and `shift` (the hit point in the current frame).
__global__ void __launch_bounds__(kWG) k_closest(const HitRec* __restrict__ hits, EvView vw,
                                                 EventState* __restrict__ ev) {
  const int e = blockIdx.y;
  if (ev[e].done) return;
  hits += vw.beg(e);
  const int32_t n_hits = vw.count(e);
  double p[5];
  for (int j = 0; j < 5; ++j) p[j] = ev[e].p[j];
  double gb = 0.0;
  int32_t ib = -1;
  for (int32_t i = threadIdx.x; i < n_hits; i += kWG) {
    if (!hits[i].use) continue;
    const double g = fabs(point_G(hits[i], p));
    if (ib < 0 || g < gb) { gb = g; ib = i; }
  }
  __shared__ double sg[kWG];
  __shared__ int32_t si[kWG];
  sg[threadIdx.x] = gb;
  si[threadIdx.x] = ib;
  __syncthreads();
  for (int w = kWG / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      const int32_t o = si[threadIdx.x + w];
      const double go = sg[threadIdx.x + w];
      const int32_t m = si[threadIdx.x];
      if (o >= 0 && (m < 0 || go < sg[threadIdx.x] || (go == sg[threadIdx.x] && o < m))) {
        sg[threadIdx.x] = go;
        si[threadIdx.x] = o;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int32_t b = si[0];
    ev[e].moving = b >= 0 ? 1 : 0;
    if (b >= 0) {
      ev[e].shift[0] = hits[b].px;
      ev[e].shift[1] = hits[b].py;
    }
  }
}

// Per-level hit selection (Sec. 3.3): after a level, every active hit of the
// pass is tested against the level's hit-finding box (estimate +- scale x
// error, in the level's frame, with the forward-hit test while the frame is
// the origin's); the hits that vote for it vote at the next level, the others
// (use = 3) sit it out.
__global__ void __launch_bounds__(kWG) k_hit_select(HitRec* __restrict__ hits, EvView vw,
                                                    const EventState* __restrict__ ev, double scale,
                                                    int32_t fwd) {
  const int e = blockIdx.y;
  if (ev[e].done) return;
  hits += vw.beg(e);
  const int32_t n_hits = vw.count(e);
  BoxD E;
  for (int j = 0; j < 5; ++j) {
    const double w = scale * ev[e].err[j];
    E.lo[j] = ev[e].p[j] - w;
    E.hi[j] = ev[e].p[j] + w;
  }
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_hits; i += stride) {
    HitRec& h = hits[i];
    if (!(h.use & 1)) continue;
    h.use = pair_vote_box(E, h, (fwd & 1) && !ev[e].moved, (fwd & 2) != 0) ? 1 : 3;
  }
}

// corner c of a box (bit j: upper end of dimension j)
IA_HD void box_corner(const BoxD& b, int c, double* x) {
  for (int j = 0; j < 5; ++j) x[j] = ((c >> j) & 1) ? b.hi[j] : b.lo[j];
}

// Extent of the boxes within `drop` votes of the maximum, over the level's
// live vote tiles (live_list, ev->n_live; every box with votes written lies
// in one): gridDim.x workgroups per event take every gridDim.x-th live tile,
// and each writes one record (minima at q = 5..9, maxima at q = 10..14).  When the event's reference point moves (move_now and
// `moving`): the hull of their 32 corners taken to the new reference point,
// phi0 unwrapped into half a turn of the first max-vote box's first corner;
// otherwise the union of the boxes, phi0 shifted by a turn where the box
// centre is more than half a turn from the first max-vote box's centre.
// Minima and maxima do not depend on the order of reduction.
__global__ void __launch_bounds__(kWG) k_window_partial(const BoxD* __restrict__ parents, Shape sh,
                                                        const uint16_t* __restrict__ votes,
                                                        const BoxD* __restrict__ first_box,
                                                        const uint16_t* __restrict__ first_votes,
                                                        double* __restrict__ part, EvView vw,
                                                        const EventState* __restrict__ ev,
                                                        const int32_t* __restrict__ wg_max,
                                                        const int32_t* __restrict__ live_list, int32_t bx,
                                                        int32_t drop, int32_t move_now) {
  const int e = blockIdx.y;
  if (ev[e].done) return;
  const bool mv = move_now && ev[e].moving;
  parents += e * vw.par_stride;
  votes += int64_t(e) * sh.n_boxes;
  wg_max += int64_t(e) * vw.wg_stride;
  live_list += int64_t(e) * vw.wg_stride;
  const int32_t n_live = ev[e].n_live;
  first_box += int64_t(e) * vw.k;
  first_votes += int64_t(e) * vw.k;
  part += int64_t(e) * vw.part_stride;
  __shared__ double sw[kWG / 64][10];
  const int32_t vlo = max(static_cast<int32_t>(first_votes[0]) - drop, 0);
  const int32_t ra = ev[e].run_a, rb = ev[e].run_b;
  const double dx = ev[e].shift[0], dy = ev[e].shift[1];
  double cref = 0.5 * (first_box->lo[1] + first_box->hi[1]);
  if (mv) {
    double x[5], q[5];
    box_corner(*first_box, 0, x);
    frame_shift(x, dx, dy, q);
    cref = q[1];
  }
  // the window is one parent box: the child widths once (child_edge's values)
  const BoxD P = parents[0];
  double w[5];
  for (int j = 0; j < 5; ++j) w[j] = (P.hi[j] - P.lo[j]) / static_cast<double>(sh.m[j]);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  // each lane keeps running extrema over the workgroup's chunks; one
  // reduction at the end writes the workgroup's record part[blockIdx.x]
  double vl[5], vh[5];
  for (int j = 0; j < 5; ++j) { vl[j] = INFINITY; vh[j] = -INFINITY; }
  // moving window: the transverse corners of each (d0, phi0, kappa) triple
  // of a tile, shifted once into the new frame (d1, phi1, arc) and shared
  // by the triple's boxes (the boxes of a triple differ only in z0, tanl)
  __shared__ double scorner[kWG][3];
  const uint32_t m34 = sh.m[3] * sh.m[4];
  const uint32_t ubx = static_cast<uint32_t>(bx);
  const bool table = mv && (ubx / m34 + 2) * 8 <= static_cast<uint32_t>(kWG);
  for (int32_t li = blockIdx.x; li < n_live; li += gridDim.x) {
    const uint32_t tile = static_cast<uint32_t>(live_list[li]);
    if (wg_max[tile] < vlo) continue;   // uniform over the workgroup
    const uint32_t b0 = tile * ubx;
    const uint32_t i = b0 + threadIdx.x;
    const bool in_set = threadIdx.x < ubx && i < sh.n_boxes && votes[i] >= vlo && in_run(phi_bin(sh, i), ra, rb);
    const uint32_t t_first = b0 / m34;
    if (table) {
      if (!__syncthreads_or(in_set ? 1 : 0)) continue;
      const uint32_t t_last = (min(b0 + ubx, sh.n_boxes) - 1) / m34;
      const uint32_t n_c = (t_last - t_first + 1) * 8;
      for (uint32_t cidx = threadIdx.x; cidx < n_c; cidx += kWG) {
        uint32_t kt[5];
        child_index(sh.m, ((t_first + cidx / 8) * m34) % sh.nc, kt);
        const int c = static_cast<int>(cidx % 8);
        double cl[3];
        for (int j = 0; j < 3; ++j) {
          const bool up = (c >> j) & 1;
          const uint32_t kk = kt[j] + (up ? 1u : 0u);
          cl[j] = (up && kk == sh.m[j]) ? P.hi[j] : P.lo[j] + static_cast<double>(kk) * w[j];
        }
        double d1, f1, arc;
        frame_shift_t(cl[0], cl[1], cl[2], dx, dy, &d1, &f1, &arc);
        const double dv = f1 - cref;
        if (dv > kPi) f1 -= kTwoPi;
        else if (dv <= -kPi) f1 += kTwoPi;
        scorner[cidx][0] = d1;
        scorner[cidx][1] = f1;
        scorner[cidx][2] = arc;
      }
      __syncthreads();
    }
    if (in_set) {
      uint32_t k[5];
      child_index(sh.m, i % sh.nc, k);
      double lo[5], hi[5];
      for (int j = 0; j < 5; ++j) {
        lo[j] = P.lo[j] + static_cast<double>(k[j]) * w[j];
        hi[j] = (k[j] + 1 == sh.m[j]) ? P.hi[j] : P.lo[j] + static_cast<double>(k[j] + 1) * w[j];
      }
      if (!mv) {
        const double dv = 0.5 * (lo[1] + hi[1]) - cref;
        double shift = 0.0;
        if (dv > kPi) shift = -kTwoPi;
        else if (dv <= -kPi) shift = kTwoPi;
        lo[1] = lo[1] + shift;
        hi[1] = hi[1] + shift;
        for (int j = 0; j < 5; ++j) { vl[j] = fmin(vl[j], lo[j]); vh[j] = fmax(vh[j], hi[j]); }
      } else {
        // the 32 corners: the transverse part of each of the 8 (d0, phi0,
        // kappa) corners once, then z0 + tanl x arc for its 4 (z0, tanl) corners
        const uint32_t tl = i / m34 - t_first;
        for (int c = 0; c < 8; ++c) {
          const double kk = (c & 4) ? hi[2] : lo[2];
          double d1, f1, arc;
          if (table) {
            d1 = scorner[tl * 8 + c][0];
            f1 = scorner[tl * 8 + c][1];
            arc = scorner[tl * 8 + c][2];
          } else {
            const double d0 = (c & 1) ? hi[0] : lo[0], f0 = (c & 2) ? hi[1] : lo[1];
            frame_shift_t(d0, f0, kk, dx, dy, &d1, &f1, &arc);
            const double dv = f1 - cref;
            if (dv > kPi) f1 -= kTwoPi;
            else if (dv <= -kPi) f1 += kTwoPi;
          }
          vl[0] = fmin(vl[0], d1); vh[0] = fmax(vh[0], d1);
          vl[1] = fmin(vl[1], f1); vh[1] = fmax(vh[1], f1);
          vl[2] = fmin(vl[2], kk); vh[2] = fmax(vh[2], kk);
          for (int zc = 0; zc < 4; ++zc) {
            const double z1 = ((zc & 1) ? hi[3] : lo[3]) + ((zc & 2) ? hi[4] : lo[4]) * arc;
            vl[3] = fmin(vl[3], z1); vh[3] = fmax(vh[3], z1);
          }
        }
        vl[4] = fmin(vl[4], lo[4]);
        vh[4] = fmax(vh[4], hi[4]);
      }
    }
  }
  // minima and maxima: across the wave with shuffles, then across waves
  for (int j = 0; j < 5; ++j)
    for (int o = 32; o > 0; o >>= 1) {
      vl[j] = fmin(vl[j], __shfl_xor(vl[j], o, 64));
      vh[j] = fmax(vh[j], __shfl_xor(vh[j], o, 64));
    }
  if (lane == 0)
    for (int j = 0; j < 5; ++j) { sw[wave][j] = vl[j]; sw[wave][5 + j] = vh[j]; }
  __syncthreads();
  if (threadIdx.x < kEstQ) {
    const int q = static_cast<int>(threadIdx.x);
    double r = 0.0;
    if (q >= 5 && q < 15) {
      const int j = q - 5;
      r = sw[0][j];
      for (int wv = 1; wv < kWG / 64; ++wv) r = j < 5 ? fmin(r, sw[wv][j]) : fmax(r, sw[wv][j]);
    }
    part[blockIdx.x * kEstQ + q] = r;
  }
}

// phi0 bins holding max-vote boxes: one bit per bin in the event state
// (chunks as k_est_partial)
__global__ void __launch_bounds__(kWG) k_phi_occ(const uint16_t* __restrict__ votes, Shape sh,
                                                 const uint16_t* __restrict__ first_votes, EventState* __restrict__ ev,
                                                 EvView vw, const int32_t* __restrict__ wg_max, int32_t bx,
                                                 uint32_t n_part, uint32_t per) {
  const int e = blockIdx.y;
  if (ev[e].done || sh.m[1] > kRunMaxBins) return;
  votes += int64_t(e) * sh.n_boxes;
  wg_max += int64_t(e) * vw.wg_stride;
  __shared__ uint32_t socc[kRunMaxBins / 32];
  if (threadIdx.x < kRunMaxBins / 32) socc[threadIdx.x] = 0u;
  __syncthreads();
  const int32_t vmax = first_votes[int64_t(e) * vw.k];
  const uint32_t ch_end = min(n_part, (blockIdx.x + 1) * per);
  __shared__ uint32_t smask;
  const uint32_t reach = chunks_reaching(wg_max, bx, blockIdx.x * per, ch_end, sh.n_boxes, vmax, &smask);
  for (uint32_t ch = blockIdx.x * per; ch < ch_end; ++ch) {
    if (!((reach >> (ch - blockIdx.x * per)) & 1u)) continue;
    const uint32_t i = ch * kWG + threadIdx.x;
    const bool at = i < sh.n_boxes && wg_max[i / static_cast<uint32_t>(bx)] >= vmax && votes[i] == vmax;
    const int32_t key = at ? static_cast<int32_t>(phi_bin(sh, i)) : -1;
    // consecutive boxes mostly share a phi0 bin: one lane sets the wave's
    // first bin for every lane holding it, the other lanes set their own
    const unsigned long long m = __ballot(at);
    if (m) {
      const int32_t k0 = __shfl(key, __ffsll(static_cast<long long>(m)) - 1, 64);
      if (key >= 0 && (key != k0 || static_cast<int32_t>(threadIdx.x & 63u) == __ffsll(static_cast<long long>(m)) - 1))
        atomicOr(&socc[key >> 5], 1u << (key & 31));
    }
  }
  __syncthreads();
  if (threadIdx.x < kRunMaxBins / 32 && socc[threadIdx.x]) atomicOr(&ev[e].occ[threadIdx.x], socc[threadIdx.x]);
}

// The run of occupied phi0 bins holding the first max-vote box's bin (one
// thread per event; circular when the level's grid spans a full turn); the
// bit mask is cleared for the next level.
__global__ void k_phi_run(const BoxD* __restrict__ parents, Shape sh, const int64_t* __restrict__ first_index,
                          EventState* __restrict__ ev, EvView vw) {
  const int e = blockIdx.y;
  if (threadIdx.x != 0 || ev[e].done) return;
  EventState& es = ev[e];
  es.run_a = -1;
  es.run_b = -1;
  const int32_t m1 = static_cast<int32_t>(sh.m[1]);
  if (sh.m[1] <= kRunMaxBins) {
    const BoxD& G = parents[e * vw.par_stride];
    const bool circ = G.hi[1] - G.lo[1] >= kTwoPi;
    auto occ = [&](int32_t k) { return (es.occ[k >> 5] >> (k & 31)) & 1u; };
    const int32_t kf = static_cast<int32_t>(phi_bin(sh, static_cast<uint32_t>(first_index[int64_t(e) * vw.k])));
    int32_t a = kf, b = kf, n = 1;
    while (n < m1) {
      int32_t k = b + 1;
      if (k == m1) { if (!circ) break; k = 0; }
      if (!occ(k)) break;
      b = k;
      ++n;
    }
    while (n < m1) {
      int32_t k = a - 1;
      if (k < 0) { if (!circ) break; k = m1 - 1; }
      if (!occ(k)) break;
      a = k;
      ++n;
    }
    if (n < m1) {
      es.run_a = a;
      es.run_b = b;
    }
  }
  for (int w = 0; w < 32; ++w) es.occ[w] = 0u;
}

struct Bins5 { int32_t m[5]; };

// Next window of an event from k_window_partial's records (one workgroup per
// event).  After a move (move_now and the event is moving): the hull of the
// corners, widened so that it spans all but one bin at each end of the next
// grid; the reference point advances by the shift.  Otherwise: the union
// widened by one of the level's bins on each side, d0 and z0 clipped to the
// range while the frame is the origin's.  Then kappa and tanl are clipped to
// the range, and a phi0 window of a full turn or more becomes the range's.
__global__ void __launch_bounds__(kWG) k_window(const double* __restrict__ part, int32_t n_part,
                                                const BoxD* __restrict__ parents, Shape sh,
                                                BoxD* __restrict__ win, EventState* __restrict__ ev, EvView vw,
                                                BoxD range, Bins5 next, int32_t move_now) {
  const int e = blockIdx.y;
  EventState& es = ev[e];
  if (es.done) return;
  part += int64_t(e) * vw.part_stride;
  const bool mv = move_now && es.moving;
  __shared__ double slo[5][kWG], shi[5][kWG];
  {
    double lo[5], hi[5];
    for (int j = 0; j < 5; ++j) { lo[j] = INFINITY; hi[j] = -INFINITY; }
    for (int32_t c = threadIdx.x; c < n_part; c += kWG)
      for (int j = 0; j < 5; ++j) {
        lo[j] = fmin(lo[j], part[c * kEstQ + 5 + j]);
        hi[j] = fmax(hi[j], part[c * kEstQ + 10 + j]);
      }
    for (int j = 0; j < 5; ++j) { slo[j][threadIdx.x] = lo[j]; shi[j][threadIdx.x] = hi[j]; }
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
      if (static_cast<int>(threadIdx.x) < w)
        for (int j = 0; j < 5; ++j) {
          slo[j][threadIdx.x] = fmin(slo[j][threadIdx.x], slo[j][threadIdx.x + w]);
          shi[j][threadIdx.x] = fmax(shi[j][threadIdx.x], shi[j][threadIdx.x + w]);
        }
      __syncthreads();
    }
  }
  if (threadIdx.x != 0) return;
  const BoxD& G = parents[e * vw.par_stride];
  BoxD nx;
  if (mv) {
    for (int j = 0; j < 5; ++j) {
      const double hl = slo[j][0], hh = shi[j][0];
      const double bin = (hh - hl) / static_cast<double>(next.m[j] > 2 ? next.m[j] - 2 : 1);
      nx.lo[j] = hl - bin;
      nx.hi[j] = hh + bin;
    }
    es.ref[0] = es.ref[0] + es.shift[0];
    es.ref[1] = es.ref[1] + es.shift[1];
    es.moved = 1;
  } else {
    for (int j = 0; j < 5; ++j) {
      const double w = (G.hi[j] - G.lo[j]) / static_cast<double>(sh.m[j]);
      nx.lo[j] = slo[j][0] - w;
      nx.hi[j] = shi[j][0] + w;
    }
    if (!es.moved)
      for (int j = 0; j < 5; j += 3) {
        nx.lo[j] = fmax(nx.lo[j], range.lo[j]);
        nx.hi[j] = fmin(nx.hi[j], range.hi[j]);
      }
  }
  for (int j = 2; j < 5; j += 2) {
    nx.lo[j] = fmax(nx.lo[j], range.lo[j]);
    nx.hi[j] = fmin(nx.hi[j], range.hi[j]);
  }
  if (nx.hi[1] - nx.lo[1] >= kTwoPi) { nx.lo[1] = range.lo[1]; nx.hi[1] = range.hi[1]; }
  win[e] = nx;
  es.moving = 0;
}

}  // namespace ia
