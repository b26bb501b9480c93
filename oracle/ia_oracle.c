/*
 * ia_oracle.c -- plain FP64 CPU oracle of the interval-arithmetic helix vote.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP library.
 *
 * Build: -O2 -ffp-contract=off -fno-fast-math.  Every interval +, -, x result
 * is computed round-to-nearest and then widened outward by
 * |x| 2^-52 + 2^-1074 (at least one ulp), so enclosures are sound and the
 * result is reproducible bit for bit; scaling by 2 or 1/2 and negation are
 * exact and not widened.  sqrt and / are the IEEE correctly rounded ones.
 * sin, cos and atan2 are written here (Cody-Waite reduction by pi/2 with a
 * three-part constant, Taylor polynomials evaluated by Horner's rule with
 * fused multiply-adds), so their results do not depend on the C library.
 *
 * Levels of a mixed-precision schedule marked FP32 use or_pair_vote32, whose
 * definition (FP32 arithmetic for the (z0, tanl) part of d^Ax, an FP32
 * interval test with a widened band) is stated at its source below.
 *
 * Parity status of each function is stated at its definition.
 */
#include "ia_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* pi/2 split for Cody-Waite reduction: the first two parts carry 33
 * significant bits, so k * part is exact for |k| < 2^20. */
static const double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
static const double PIO2_1 = 0x1.921fb544p+0;
static const double PIO2_2 = 0x1.0b4611a6p-34;
static const double PIO2_3 = 0x1.3198a2e037073p-69;
static const double PI_RN = 0x1.921fb54442d18p+1;      /* pi, rounded (below pi) */
static const double TWO_PI_RN = 0x1.921fb54442d18p+2;  /* 2 pi, rounded (below 2 pi) */
static const double PIO2_RN = 0x1.921fb54442d18p+0;
static const double PIO2_UP = 0x1.921fb54442d19p+0;   /* pi/2 rounded up */
static const double PIO6_RN = 0x1.0c152382d7366p-1;
static const double SQRT3_RN = 0x1.bb67ae8584caap+0;
static const double INV_TWO_PI = 0x1.45f306dc9c883p-3;
static const double TAN_PI_12 = 0x1.126145e9ecd56p-2;  /* 2 - sqrt(3) */
static const double SIN_MARGIN = 0x1p-50;  /* > 4x the measured error of or_sin */
static const double EXT_FUZZ = 0x1p-40;    /* slack of the extremum test */

/* ------------------------------------------------------------------------
 * elementary functions (pinned against mpmath in the tests)
 * ---------------------------------------------------------------------- */
/* sin r on |r| <= pi/4: Taylor series to degree 17, coefficients 1/n! */
static double sin_poly(double r) {
  double z = r * r;
  double p = 1.0 / 355687428096000.0;
  p = fma(p, z, -1.0 / 1307674368000.0);
  p = fma(p, z, 1.0 / 6227020800.0);
  p = fma(p, z, -1.0 / 39916800.0);
  p = fma(p, z, 1.0 / 362880.0);
  p = fma(p, z, -1.0 / 5040.0);
  p = fma(p, z, 1.0 / 120.0);
  p = fma(p, z, -1.0 / 6.0);
  return fma(r * z, p, r);
}

/* cos r on |r| <= pi/4: Taylor series to degree 16 */
static double cos_poly(double r) {
  double z = r * r;
  double q = 1.0 / 20922789888000.0;
  q = fma(q, z, -1.0 / 87178291200.0);
  q = fma(q, z, 1.0 / 479001600.0);
  q = fma(q, z, -1.0 / 3628800.0);
  q = fma(q, z, 1.0 / 40320.0);
  q = fma(q, z, -1.0 / 720.0);
  q = fma(q, z, 1.0 / 24.0);
  q = fma(q, z, -0.5);
  return fma(z, q, 1.0);
}

/* x = k pi/2 + r with |r| <= pi/4 (plus rounding) */
static double reduce_pio2(double x, int64_t *k_out) {
  double k = rint(x * TWO_OVER_PI);
  double r = ((x - k * PIO2_1) - k * PIO2_2) - k * PIO2_3;
  *k_out = (int64_t)k;
  return r;
}

double or_sin(double x) {
  int64_t k;
  double r = reduce_pio2(x, &k);
  switch (k & 3) {
    case 0: return sin_poly(r);
    case 1: return cos_poly(r);
    case 2: return -sin_poly(r);
    default: return -cos_poly(r);
  }
}

double or_cos(double x) {
  int64_t k;
  double r = reduce_pio2(x, &k);
  switch (k & 3) {
    case 0: return cos_poly(r);
    case 1: return -sin_poly(r);
    case 2: return -cos_poly(r);
    default: return sin_poly(r);
  }
}

/* atan u on |u| <= tan(pi/12): Taylor series to degree 29 */
static double atan_poly(double u) {
  double z = u * u;
  double p = 1.0 / 29.0;
  p = fma(p, z, -1.0 / 27.0);
  p = fma(p, z, 1.0 / 25.0);
  p = fma(p, z, -1.0 / 23.0);
  p = fma(p, z, 1.0 / 21.0);
  p = fma(p, z, -1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, -1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, -1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, -1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, -1.0 / 3.0);
  return fma(u * z, p, u);
}

/* atan t on [0, 1]; above tan(pi/12) use atan t = pi/6 + atan((t sqrt3 - 1)/(t + sqrt3)) */
static double atan_unit(double t) {
  if (t > TAN_PI_12) return PIO6_RN + atan_poly((t * SQRT3_RN - 1.0) / (t + SQRT3_RN));
  return atan_poly(t);
}

/* the angle of (x, y), in [-pi, pi]; 0 for the origin */
double or_atan2(double y, double x) {
  double ax = fabs(x), ay = fabs(y);
  if (ax == 0.0 && ay == 0.0) return 0.0;
  int swap = ay > ax;
  double a = atan_unit(swap ? ax / ay : ay / ax);
  if (swap) a = PIO2_RN - a;
  if (x < 0.0) a = PI_RN - a;
  if (y < 0.0) a = -a;
  return a;
}

/* ------------------------------------------------------------------------
 * interval arithmetic (Moore intervals, outward rounded)
 * ---------------------------------------------------------------------- */
double or_wdn(double x) { return x - fma(fabs(x), 0x1p-52, 0x1p-1074); }
double or_wup(double x) { return x + fma(fabs(x), 0x1p-52, 0x1p-1074); }

typedef struct { double lo, hi; } iv;

static iv iv_add(iv a, iv b) { iv r = {or_wdn(a.lo + b.lo), or_wup(a.hi + b.hi)}; return r; }
static iv iv_sub(iv a, iv b) { iv r = {or_wdn(a.lo - b.hi), or_wup(a.hi - b.lo)}; return r; }
static iv iv_mul(iv a, iv b) {
  double p1 = a.lo * b.lo, p2 = a.lo * b.hi, p3 = a.hi * b.lo, p4 = a.hi * b.hi;
  iv r = {or_wdn(fmin(fmin(p1, p2), fmin(p3, p4))), or_wup(fmax(fmax(p1, p2), fmax(p3, p4)))};
  return r;
}
static iv iv_sqr(iv a) {
  double l2 = a.lo * a.lo, h2 = a.hi * a.hi;
  iv r;
  if (a.lo <= 0.0 && a.hi >= 0.0) { r.lo = 0.0; r.hi = or_wup(fmax(l2, h2)); }
  else { r.lo = or_wdn(fmin(l2, h2)); r.hi = or_wup(fmax(l2, h2)); }
  return r;
}
static iv iv_twice(iv a) { iv r = {2.0 * a.lo, 2.0 * a.hi}; return r; }
static iv iv_point(double x) { iv r = {x, x}; return r; }

void or_imul(double alo, double ahi, double blo, double bhi, double *lo, double *hi) {
  iv a = {alo, ahi}, b = {blo, bhi}, r = iv_mul(a, b);
  *lo = r.lo; *hi = r.hi;
}
void or_isqr(double alo, double ahi, double *lo, double *hi) {
  iv a = {alo, ahi}, r = iv_sqr(a);
  *lo = r.lo; *hi = r.hi;
}

/* Enclosure of sin over [a, b].  Between extrema sin is monotone, so the end
 * values (less / plus a margin above the error of or_sin) bound it; an
 * interval that may contain pi/2 + 2k pi (resp. -pi/2 + 2k pi) gets hi = 1
 * (resp. lo = -1).  The membership test is fuzzed by 2^-40 so that rounding
 * can only make it answer "contains". */
void or_sin_encl(double a, double b, double *lo, double *hi) {
  if (b - a >= TWO_PI_RN) { *lo = -1.0; *hi = 1.0; return; }
  double va = or_sin(a), vb = or_sin(b);
  double l = fmin(va, vb) - SIN_MARGIN, h = fmax(va, vb) + SIN_MARGIN;
  if (floor((b - PIO2_RN) * INV_TWO_PI + EXT_FUZZ) >= ceil((a - PIO2_RN) * INV_TWO_PI - EXT_FUZZ)) h = 1.0;
  if (floor((b + PIO2_RN) * INV_TWO_PI + EXT_FUZZ) >= ceil((a + PIO2_RN) * INV_TWO_PI - EXT_FUZZ)) l = -1.0;
  if (l < -1.0) l = -1.0;
  if (h > 1.0) h = 1.0;
  *lo = l; *hi = h;
}

/* ------------------------------------------------------------------------
 * hit preparation: the wire point at z = 0 and the stereo direction
 * (Eqs. wirePar_a,b; Eqs. EQSinter_d,e with z_ref = 0)
 * ---------------------------------------------------------------------- */
int32_t or_prep_hit(const or_hit *h, or_prep *o) { return or_prep_hit_ref(h, 0.0, 0.0, o); }

/* The paper moves the reference point of the parametrisation near the hits
 * between iterations (Sec. 3.3).  Perigee parameters about a reference point
 * a are those of the hits translated by -a, so the hit point is taken about
 * a: (px - xr, py - yr), one rounding each (exact for a = 0). */
int32_t or_prep_hit_ref(const or_hit *h, double xr, double yr, or_prep *o) {
  memset(o, 0, sizeof *o);
  const double *f = &h->x0;
  for (int i = 0; i < 8; i++) if (!isfinite(f[i])) return 0;
  double dz = h->z1 - h->z0;
  if (dz == 0.0 || h->drift < 0.0 || h->band < 0.0) return 0;
  double tx = (h->x1 - h->x0) / dz, ty = (h->y1 - h->y0) / dz;
  o->px = (h->x0 - h->z0 * tx) - xr;
  o->py = (h->y0 - h->z0 * ty) - yr;
  o->tant = sqrt(tx * tx + ty * ty);
  if (!isfinite(o->px) || !isfinite(o->py) || !isfinite(o->tant)) return 0;
  /* direction (sin phi_s, -cos phi_s) tan(tau) = (tx, ty) with tan(tau) >= 0 */
  if (o->tant == 0.0) { o->sphis = 0.0; o->cphis = 1.0; o->axial = 1; }
  else { o->sphis = tx / o->tant; o->cphis = -ty / o->tant; o->axial = 0; }
  o->r = sqrt(o->px * o->px + o->py * o->py);
  o->phip = or_atan2(o->py, o->px);
  double r2 = o->r * o->r;
  o->r2lo = or_wdn(r2);
  o->r2hi = or_wup(r2);
  o->d = h->drift;
  o->band = h->band;
  o->valid = 1;
  return 1;
}

/* ------------------------------------------------------------------------
 * boxes: regular split of a parent box (edges L + k w, last edge U)
 * ---------------------------------------------------------------------- */
void or_box_child(const or_box *par, const int32_t m[5], int64_t child, or_box *out) {
  int64_t k[5], rem = child;
  for (int j = 4; j >= 0; j--) { k[j] = rem % m[j]; rem /= m[j]; }
  for (int j = 0; j < 5; j++) {
    double L = par->lo[j], U = par->hi[j], w = (U - L) / (double)m[j];
    out->lo[j] = L + (double)k[j] * w;
    out->hi[j] = (k[j] + 1 == m[j]) ? U : L + (double)(k[j] + 1) * w;
  }
}

/* ------------------------------------------------------------------------
 * virtual drift distance d^Ax at a point of parameter space
 * (Appendix A: Eqs. normudi, EQSinter_c, defdiAX_b, CSAXtoPHI_a's
 * definitions and the second-order solution ApproxPhi, with z_ref = 0).
 *
 * Appendix A assumes R > 0.  A point with kappa < 0 is mirrored (y -> -y),
 * which maps the helix to one with kappa > 0, d0 -> -d0, phi0 -> -phi0 and the
 * wire to its mirror image; d^Ax is computed there and returned as
 * e = sgn(kappa) d^Ax, the drift term of the kappa-scaled residual.
 * ---------------------------------------------------------------------- */
/* the quantities of the stereo point for a given Phi - Phi^Ax = eps
 * (Eqs. normudi, EQSinter_c, c^tau and s^tau of Appendix A) */
typedef struct { double sinP, cosP, u, delta, sperp, zS, ld, ctau, stau; } st_point;

static st_point stereo_point(double eps, double sinA, double cosA, double lam, double tt, double t2, double dS,
                             double R, double dphi, double z0, double cAx, double sAx) {
  st_point q;
  double se = or_sin(eps), ce = or_cos(eps);
  q.sinP = sinA * ce + cosA * se;
  q.cosP = cosA * ce - sinA * se;
  q.u = sqrt(((1.0 + ((2.0 * lam) * q.sinP) * tt) + (lam * lam) * t2) + (q.cosP * q.cosP) * t2);
  q.delta = dS / q.u;
  q.sperp = R * (dphi + eps);                 /* rho s_perp = Phi + phi_s - phi0 */
  q.zS = (z0 + lam * q.sperp) - (q.delta * q.cosP) * tt;   /* z_i^St (EQSinter_c) */
  q.ld = lam * q.delta;
  q.ctau = q.zS * cAx - q.ld * sAx;           /* c_i^tau */
  q.stau = -(q.ld * cAx + q.zS * sAx);        /* s_i^tau */
  return q;
}

int32_t or_stereo_e(const or_prep *h, const double c[5], int32_t s, double *e, double *dbg) {
  return or_stereo_e_x(h, c, s, 0, e, dbg);
}

/* exact = 1: Phi solves Eq. CSAXtoPHI_a, Phi = Phi^Ax + atan2(s^tau tan(tau),
 * (R^Ax)^2 + c^tau tan(tau)), by OR_PHI_ITERS fixed-point steps started from
 * the second-order solution ApproxPhi (the map contracts by about
 * |tan(tau) tanl| R / R^Ax per step, and d^Ax is stationary in Phi at the
 * closest approach, so its error falls as the square of Phi's).  With the
 * exact Phi the closest approach does not depend on z_ref, which therefore
 * stays 0. */
int32_t or_stereo_e_x(const or_prep *h, const double c[5], int32_t s, int32_t exact, double *e, double *dbg) {
  double kap = c[2], sig = 1.0;
  if (kap < 0.0) sig = -1.0;
  if (kap == 0.0) { kap = 0x1p-30; sig = 1.0; }
  double dS = (double)s * h->d;               /* signed drift d^St */
  if (h->axial) {                             /* tan(tau) = 0: d^Ax = d^St */
    *e = sig * dS;
    return 1;
  }
  double kp = sig * kap, d0p = sig * c[0];
  double sp0 = sig * or_sin(c[1]), cp0 = or_cos(c[1]);
  double R = 1.0 / kp;
  double Rd = R + d0p;
  double xc = -(Rd * sp0), yc = Rd * cp0;     /* circle centre (HelixEq_d) */
  double py = sig * h->py, cps = sig * h->cphis, sps = h->sphis;
  double Dx = h->px - xc, Dy = py - yc;
  double RAx = sqrt(Dx * Dx + Dy * Dy);       /* R_i^Ax */
  double cAx = Dx * sps - Dy * cps;           /* c_i^Ax */
  double sAx = Dx * cps + Dy * sps;           /* s_i^Ax */
  double sinA = sAx / RAx, cosA = cAx / RAx;  /* sin, cos of Phi_i^Ax */
  /* phi_i^Ax - phi0, wrapped to [-pi, pi] */
  double dphi = or_atan2(Dx * cp0 + Dy * sp0, Dx * sp0 - Dy * cp0);
  double z0 = c[3], lam = c[4], tt = h->tant;
  double sArc = R * dphi;                     /* transverse arc length to the axial point */
  double zA = z0 + lam * sArc;                /* z_i^Ax (ApproxPhi_d) */
  /* first- and second-order terms of Phi_i (ApproxPhi_b, ApproxPhi_c) */
  double Phi1 = -(zA * sinA + (lam * dS) * cosA) / RAx;
  double c2 = cosA * cosA - sinA * sinA;      /* cos 2 Phi^Ax */
  double s2 = 2.0 * sinA * cosA;              /* sin 2 Phi^Ax */
  double Phi2n = (lam * R) * zA - ((lam * zA) * (R - 2.0 * dS)) * c2
               + (zA * zA + dS * (RAx + (lam * lam) * ((R + RAx) - dS))) * s2;
  double Phi2 = Phi2n / (2.0 * (RAx * RAx));
  double t2 = tt * tt;
  double eps = Phi1 * tt + Phi2 * t2;         /* Phi_i - Phi_i^Ax (ApproxPhi) */
  if (exact) {
    double RAx2 = RAx * RAx;
    for (int k = 0; k < OR_PHI_ITERS; k++) {
      st_point q = stereo_point(eps, sinA, cosA, lam, tt, t2, dS, R, dphi, z0, cAx, sAx);
      eps = or_atan2(q.stau * tt, RAx2 + q.ctau * tt);
    }
  }
  st_point q = stereo_point(eps, sinA, cosA, lam, tt, t2, dS, R, dphi, z0, cAx, sAx);
  double sinP = q.sinP, cosP = q.cosP, u = q.u, delta = q.delta, sperp = q.sperp, zS = q.zS, ctau = q.ctau;
  double a1 = zS * tt, a2 = q.ld * tt;
  double Q = ((2.0 * ctau) * tt + a1 * a1) + a2 * a2;
  double A = R + delta;
  double disc = A * A - Q;
  if (!(disc >= 0.0)) return 0;
  /* d^Ax = sqrt((R + delta)^2 - Q) - R  (defdiAX_b), written without cancellation */
  double dhat = delta - Q / (A + sqrt(disc));
  if (dbg) {
    double v[24] = {R, xc, yc, Dx, Dy, RAx, cAx, sAx, sinA, cosA, dphi, zA, Phi1, Phi2,
                    eps, sinP, cosP, u, delta, sperp, zS, ctau, Q, dhat};
    memcpy(dbg, v, sizeof v);
  }
  *e = sig * dhat;
  return isfinite(*e) ? 1 : 0;
}

/* ------------------------------------------------------------------------
 * the vote predicate, Eq. ApoVote, multiplied by kappa:
 *   kappa F = 2 G - 2 e - kappa e^2,
 *   G = (kappa/2)(r^2 + d0^2) + (1 + kappa d0) r sin(phi0 - phiP) + d0,
 * which is kappa (|P - C|^2 - R^2) / 2 in perigee variables.  G is enclosed
 * over the whole box; e is the point value at the middle of the box for each
 * drift sign; one vote when zero is enclosed for either sign.
 * ---------------------------------------------------------------------- */
static iv pair_G(const or_prep *h, const or_box *b) {
  iv K = {b->lo[2], b->hi[2]}, Dd = {b->lo[0], b->hi[0]};
  iv Ar = {or_wdn(b->lo[1] - h->phip), or_wup(b->hi[1] - h->phip)};
  iv S;
  or_sin_encl(Ar.lo, Ar.hi, &S.lo, &S.hi);
  iv rS = iv_mul(S, iv_point(h->r));
  iv D2 = iv_sqr(Dd);
  iv T0 = iv_add(D2, (iv){h->r2lo, h->r2hi});
  iv T = {0.5 * T0.lo, 0.5 * T0.hi};
  iv KT = iv_mul(K, T);
  iv KD1 = iv_add(iv_mul(K, Dd), iv_point(1.0));
  return iv_add(iv_add(KT, iv_mul(KD1, rS)), Dd);
}

int32_t or_pair_vote(const or_prep *h, const or_box *b, double *dbg) {
  return or_pair_vote_x(h, b, 0, dbg);
}

int32_t or_pair_vote_x(const or_prep *h, const or_box *b, int32_t exact, double *dbg) {
  if (!h->valid) return 0;
  iv K = {b->lo[2], b->hi[2]};
  iv G = pair_G(h, b);
  double c[5];
  for (int j = 0; j < 5; j++) c[j] = 0.5 * (b->lo[j] + b->hi[j]);
  int32_t vote = 0;
  if (dbg) { dbg[0] = G.lo; dbg[1] = G.hi; for (int j = 2; j < 8; j++) dbg[j] = NAN; }
  for (int32_t si = 0; si < 2; si++) {
    int32_t s = si == 0 ? 1 : -1;
    double e;
    if (!or_stereo_e_x(h, c, s, exact, &e, NULL)) continue;
    iv E = {or_wdn(e - h->band), or_wup(e + h->band)};
    iv H = iv_sub(iv_twice(G), iv_add(iv_twice(E), iv_mul(K, iv_sqr(E))));
    if (dbg) { dbg[2 + 2 * si] = H.lo; dbg[3 + 2 * si] = H.hi; dbg[6 + si] = e; }
    if (H.lo <= 0.0 && 0.0 <= H.hi) vote = 1;
  }
  return vote;
}

/* ------------------------------------------------------------------------
 * Sound d^Ax over a whole box (IV levels).  Sec. 3.1 takes d^Ax at the
 * middle of the voxel, which the paper notes is not an enclosure.  Here
 * every quantity of Appendix A is enclosed over the whole box in interval
 * arithmetic (outward rounding as above), in the kappa > 0 frame of the
 * box (a box whose kappa range holds 0 has no such frame: no enclosure):
 * the circle centre and radius, R^Ax, c^Ax, s^Ax, sin and cos Phi^Ax,
 * phi^Ax - phi0 (atan2 enclosed by its values at the corners of its
 * argument box plus 1e-13, or [-pi, pi] where that box meets the cut), then
 * Phi itself: Phi - Phi^Ax solves Eq. CSAXtoPHI_a, eps = atan2(s^tau tan
 * tau, (R^Ax)^2 + c^tau tan tau), so every solution lies in F(EPS) for any
 * EPS that holds it, F the interval image of the right-hand side.  Starting
 * from [-pi, pi] (where the denominator must stay positive, else no
 * enclosure), OR_IV_ITERS steps EPS <- EPS meet F(EPS) keep every solution,
 * hence the exact closest approach, for every point of the box.  With EPS,
 * Eqs. normudi, EQSinter_c and defdiAX_b in interval form give d^Ax; the
 * enclosure is returned for e = sgn(kappa) d^Ax.
 * Parity: pinned by sampled points of random boxes, whose exact-Phi point
 * values (themselves pinned against the generator's closest approach) lie
 * inside, and by the vote containing the mid-voxel vote's hits at the truth.
 * ---------------------------------------------------------------------- */
static iv iv_neg(iv a) { iv r = {-a.hi, -a.lo}; return r; }
static iv iv_mulp(iv a, double x) {
  double p = a.lo * x, q = a.hi * x;
  iv r;
  if (x >= 0.0) { r.lo = or_wdn(p); r.hi = or_wup(q); } else { r.lo = or_wdn(q); r.hi = or_wup(p); }
  return r;
}
/* a / b for b.lo > 0 */
static iv iv_divpos(iv a, iv b) {
  double q1 = a.lo / b.lo, q2 = a.lo / b.hi, q3 = a.hi / b.lo, q4 = a.hi / b.hi;
  iv r = {or_wdn(fmin(fmin(q1, q2), fmin(q3, q4))), or_wup(fmax(fmax(q1, q2), fmax(q3, q4)))};
  return r;
}
static iv iv_sqrt(iv a) { iv r = {a.lo > 0.0 ? or_wdn(sqrt(a.lo)) : 0.0, or_wup(sqrt(a.hi))}; return r; }
static iv iv_sin(iv a) { iv r; or_sin_encl(a.lo, a.hi, &r.lo, &r.hi); return r; }
static iv iv_cos(iv a) {
  iv r;
  or_sin_encl(or_wdn(a.lo + PIO2_RN), or_wup(a.hi + PIO2_UP), &r.lo, &r.hi);
  return r;
}
static iv iv_atan2(iv y, iv x) {
  if (x.lo <= 0.0 && y.lo <= 0.0 && y.hi >= 0.0) { iv r = {-2.0 * PIO2_UP, 2.0 * PIO2_UP}; return r; }
  double a = or_atan2(y.lo, x.lo), b = or_atan2(y.lo, x.hi), c = or_atan2(y.hi, x.lo), d = or_atan2(y.hi, x.hi);
  iv r = {fmin(fmin(a, b), fmin(c, d)) - 1e-13, fmax(fmax(a, b), fmax(c, d)) + 1e-13};
  return r;
}

typedef struct { iv sinP, cosP, u, delta, zS, ld, ctau; } iv_stpoint;

/* the stereo-point quantities for Phi - Phi^Ax in EPS; 0 when u^2 may be <= 0 */
static int32_t iv_stereo_point(iv EPS, iv SINA, iv COSA, iv LAM, double tt, iv T2, double dS, iv R, iv DPHI,
                               iv Z0, iv CAX, iv SAX, iv_stpoint *o) {
  iv SE = iv_sin(EPS), CE = iv_cos(EPS);
  o->sinP = iv_add(iv_mul(SINA, CE), iv_mul(COSA, SE));
  o->cosP = iv_sub(iv_mul(COSA, CE), iv_mul(SINA, SE));
  iv U2 = iv_add(iv_add(iv_add(iv_point(1.0), iv_mulp(iv_mul(iv_twice(LAM), o->sinP), tt)),
                        iv_mul(iv_sqr(LAM), T2)),
                 iv_mul(iv_sqr(o->cosP), T2));
  if (!(U2.lo > 0.0)) return 0;
  o->u = iv_sqrt(U2);
  o->delta = iv_divpos(iv_point(dS), o->u);
  iv SPERP = iv_mul(R, iv_add(DPHI, EPS));
  o->zS = iv_sub(iv_add(Z0, iv_mul(LAM, SPERP)), iv_mulp(iv_mul(o->delta, o->cosP), tt));
  o->ld = iv_mul(LAM, o->delta);
  o->ctau = iv_sub(iv_mul(o->zS, CAX), iv_mul(o->ld, SAX));
  return 1;
}

int32_t or_stereo_encl(const or_prep *h, const or_box *b, int32_t s, double *lo, double *hi) {
  if (!h->valid) return 0;
  if (b->lo[2] <= 0.0 && b->hi[2] >= 0.0) return 0;            /* kappa of both signs */
  const double sig = b->lo[2] > 0.0 ? 1.0 : -1.0;
  const iv K = {b->lo[2], b->hi[2]}, D0 = {b->lo[0], b->hi[0]}, FI = {b->lo[1], b->hi[1]};
  const double dS = (double)s * h->d;
  if (h->axial) {                                               /* tan(tau) = 0: d^Ax = d^St */
    *lo = sig * dS;
    *hi = sig * dS;
    return 1;
  }
  const iv KP = sig > 0.0 ? K : iv_neg(K), D0P = sig > 0.0 ? D0 : iv_neg(D0);
  const iv SF = iv_sin(FI), CP0 = iv_cos(FI);
  const iv SP0 = sig > 0.0 ? SF : iv_neg(SF);
  const iv R = {or_wdn(1.0 / KP.hi), or_wup(1.0 / KP.lo)};
  const iv RD = iv_add(R, D0P);
  const iv XC = iv_neg(iv_mul(RD, SP0)), YC = iv_mul(RD, CP0);
  const double py = sig * h->py, cps = sig * h->cphis, sps = h->sphis;
  const iv DX = iv_sub(iv_point(h->px), XC), DY = iv_sub(iv_point(py), YC);
  const iv RAX2 = iv_add(iv_sqr(DX), iv_sqr(DY));
  if (!(RAX2.lo > 0.0)) return 0;
  const iv RAX = iv_sqrt(RAX2);
  const iv CAX = iv_sub(iv_mulp(DX, sps), iv_mulp(DY, cps));
  const iv SAX = iv_add(iv_mulp(DX, cps), iv_mulp(DY, sps));
  const iv SINA = iv_divpos(SAX, RAX), COSA = iv_divpos(CAX, RAX);
  const iv YY = iv_add(iv_mul(DX, CP0), iv_mul(DY, SP0)), XX = iv_sub(iv_mul(DX, SP0), iv_mul(DY, CP0));
  const iv DPHI = iv_atan2(YY, XX);
  const iv Z0 = {b->lo[3], b->hi[3]}, LAM = {b->lo[4], b->hi[4]};
  const double tt = h->tant;
  const iv T2 = {or_wdn(tt * tt), or_wup(tt * tt)};
  /* every solution of Eq. CSAXtoPHI_a over the box */
  iv EPS = {-2.0 * PIO2_UP, 2.0 * PIO2_UP};
  iv_stpoint q;
  for (int k = 0; k < OR_IV_ITERS; k++) {
    if (!iv_stereo_point(EPS, SINA, COSA, LAM, tt, T2, dS, R, DPHI, Z0, CAX, SAX, &q)) return 0;
    const iv ST = iv_neg(iv_add(iv_mul(q.ld, CAX), iv_mul(q.zS, SAX)));
    const iv DEN = iv_add(RAX2, iv_mulp(q.ctau, tt));
    if (!(DEN.lo > 0.0)) return 0;
    const iv F = iv_atan2(iv_mulp(ST, tt), DEN);
    EPS.lo = fmax(EPS.lo, F.lo);
    EPS.hi = fmin(EPS.hi, F.hi);
    if (!(EPS.lo <= EPS.hi)) return 0;
  }
  if (!iv_stereo_point(EPS, SINA, COSA, LAM, tt, T2, dS, R, DPHI, Z0, CAX, SAX, &q)) return 0;
  const iv A1 = iv_mulp(q.zS, tt), A2 = iv_mulp(q.ld, tt);
  const iv Q = iv_add(iv_add(iv_mulp(iv_twice(q.ctau), tt), iv_sqr(A1)), iv_sqr(A2));
  const iv A = iv_add(R, q.delta);
  const iv DISC = iv_sub(iv_sqr(A), Q);
  if (!(DISC.lo > 0.0) || !(A.lo > 0.0)) return 0;
  const iv DHAT = iv_sub(q.delta, iv_divpos(Q, iv_add(A, iv_sqrt(DISC))));
  const iv E = sig > 0.0 ? DHAT : iv_neg(DHAT);
  if (!isfinite(E.lo) || !isfinite(E.hi)) return 0;
  *lo = E.lo;
  *hi = E.hi;
  return 1;
}

/* the vote of one (box, hit) at an IV level: zero in 2G - 2E - kappa E^2 for
 * either drift sign, with E the box enclosure of d^Ax widened by the band;
 * no enclosure: the pair votes */
int32_t or_pair_vote_iv(const or_prep *h, const or_box *b) {
  if (!h->valid) return 0;
  if (h->axial) return or_pair_vote(h, b, NULL);
  const iv K = {b->lo[2], b->hi[2]};
  const iv G = pair_G(h, b);
  for (int32_t si = 0; si < 2; si++) {
    double lo, hi;
    if (!or_stereo_encl(h, b, si == 0 ? 1 : -1, &lo, &hi)) return 1;
    const iv E = {or_wdn(lo - h->band), or_wup(hi + h->band)};
    const iv H = iv_sub(iv_twice(G), iv_add(iv_twice(E), iv_mul(K, iv_sqr(E))));
    if (H.lo <= 0.0 && 0.0 <= H.hi) return 1;
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Forward-hit test.  The paper's particles come from the origin (Sec. 3.2),
 * so along the direction of travel every hit lies after the point of
 * closest approach.  Without this, the perigee form holds every helix twice:
 * (d0, phi0, kappa, z0, tanl) and (-d0, phi0 + pi, -kappa, z0, -tanl) trace
 * the same points in opposite directions and get the same votes.  The hit
 * point P is ahead of the point of closest approach d0 (-sin phi0, cos phi0)
 * when (P - PCA).(cos phi0, sin phi0) = r cos(phi0 - phiP) > 0.  Over the
 * box's phi0 interval, cos(phi0 - phiP) = sin(phi0 - phiP + pi/2) is
 * enclosed with the outward sine enclosure (the shifted ends rounded outward,
 * pi/2 taken below it at the lower end and above it at the upper end); a hit
 * is ahead for some phi0 of
 * the box when the enclosure's upper end is positive (a sound test: it can
 * only answer "ahead" too often).
 * Parity: pinned by brute force over sampled phi0 and by the twin test.
 * ---------------------------------------------------------------------- */
int32_t or_forward(const or_prep *h, const or_box *b) {
  if (h->r == 0.0) return 1;
  double lo = or_wdn(or_wdn(b->lo[1] - h->phip) + PIO2_RN);
  double hi = or_wup(or_wup(b->hi[1] - h->phip) + PIO2_UP);
  double slo, shi;
  or_sin_encl(lo, hi, &slo, &shi);
  return shi > 0.0;
}

/* ------------------------------------------------------------------------
 * Change of reference point (Sec. 3.3 moves it between iterations).  The
 * circle of p about a has centre C = a + (1/kappa + d0) n with
 * n = (-sin phi0, cos phi0); about b = a + D it is C = b + (1/kappa + d0') n'.
 * Multiplying by kappa, A = (1 + kappa d0) n - kappa D = (1 + kappa d0') n',
 * so n' = A / |A|, phi0' = atan2(-A_x, A_y) and
 *   d0' = (|A|^2 - 1) / (kappa (|A| + 1))
 *       = (2 d0 + kappa d0^2 - 2 (1 + kappa d0) n.D + kappa |D|^2) / (|A| + 1),
 * which stays finite as kappa -> 0 (there d0' = d0 - n.D, a line).  The
 * direction turns by dphi = atan2(kappa u.D, 1 + kappa d0 - kappa n.D) with
 * u = (cos phi0, sin phi0) from the old point of closest approach to the
 * new one, over the arc s = dphi / kappa (s = u.D when kappa = 0), and z
 * grows by tanl s (Eq. HelixEq_c).  kappa and tanl do not change.
 * Parity: pinned against a direct closest-point computation and by the
 * round trip a -> b -> a.
 * ---------------------------------------------------------------------- */
void or_frame_shift(const double p[5], double dx, double dy, double q[5]) {
  double d0 = p[0], f0 = p[1], k = p[2], z0 = p[3], l = p[4];
  double s0 = or_sin(f0), c0 = or_cos(f0);
  double nD = -s0 * dx + c0 * dy;
  double uD = c0 * dx + s0 * dy;
  double one = 1.0 + k * d0;
  double ax = one * (-s0) - k * dx;
  double ay = one * c0 - k * dy;
  double A = sqrt(ax * ax + ay * ay);
  double num = 2.0 * d0 + k * (d0 * d0) - 2.0 * one * nD + k * (dx * dx + dy * dy);
  double f1 = or_atan2(-ax, ay);
  if (f1 < 0.0) f1 += TWO_PI_RN;
  double arc = uD;
  if (k != 0.0) arc = or_atan2(k * uD, one - k * nD) / k;
  q[0] = num / (A + 1.0);
  q[1] = f1;
  q[2] = k;
  q[3] = z0 + l * arc;
  q[4] = l;
}

/* ------------------------------------------------------------------------
 * The disk condition, Eq. ApoVoteDisk (Sec. 3.1): a voxel is considered only
 * if some circle of it passes within R_disk of the emission point, the
 * origin.  That is Eq. ApoVote for a measurement at the origin with drift
 * distance 0 and tolerance R_disk: an axial hit whose point is the origin
 * taken about the reference point.  The paper uses it to skip voxels; here
 * it also keeps the search near the origin after the reference point moves.
 * Parity: pinned on sampled circles (distance from the origin).
 * ---------------------------------------------------------------------- */
int32_t or_disk(const or_box *b, double xr, double yr, double disk) {
  or_prep h;
  memset(&h, 0, sizeof h);
  h.valid = 1;
  h.axial = 1;
  h.px = -xr;
  h.py = -yr;
  h.tant = 0.0;
  h.sphis = 0.0;
  h.cphis = 1.0;
  h.r = sqrt(h.px * h.px + h.py * h.py);
  h.phip = h.r == 0.0 ? 0.0 : or_atan2(h.py, h.px);
  double r2 = h.r * h.r;
  h.r2lo = or_wdn(r2);
  h.r2hi = or_wup(r2);
  h.d = 0.0;
  h.band = disk;
  return or_pair_vote(&h, b, NULL);
}

/* About a moved reference point the forward-hit test no longer applies (the
 * hits lie on both sides of it), and the mirror twin returns.  The track
 * still comes from the origin: the origin, seen from the point of closest
 * approach, lies behind it, r_O cos(phi0 - phi_O) < 0 with phi_O the
 * direction of the origin from the reference point.  Over the box's phi0
 * interval the lower end of the enclosure of cos(phi0 - phi_O) =
 * sin(phi0 - phi_O + pi/2) decides (outward, as in or_forward).
 * Parity: pinned by brute force over sampled phi0 and by the twin test. */
int32_t or_behind(const or_box *b, double xr, double yr) {
  if (xr == 0.0 && yr == 0.0) return 1;
  double phio = or_atan2(-yr, -xr);
  double lo = or_wdn(or_wdn(b->lo[1] - phio) + PIO2_RN);
  double hi = or_wup(or_wup(b->hi[1] - phio) + PIO2_UP);
  double slo, shi;
  or_sin_encl(lo, hi, &slo, &shi);
  return slo < 0.0;
}

/* G of Eq. ApoVote's kappa-scaled form at one parameter point */
double or_point_G(const or_prep *h, const double p[5]) {
  double d0 = p[0], k = p[2];
  return 0.5 * k * (h->r * h->r + d0 * d0) + (1.0 + k * d0) * (h->r * or_sin(p[1] - h->phip)) + d0;
}

/* ------------------------------------------------------------------------
 * FP32 levels of a mixed-precision schedule.
 *
 * The paper computes in FP64 throughout.  A level marked FP32 evaluates the
 * whole predicate of a (box, hit) pair in FP32:
 *  - the box edges enter as FP32 intervals rounded outward, the hit's
 *    prepared quantities (FP64, once per hit) rounded outward where they are
 *    intervals (r, r^2, phi_P) and to nearest where they are points;
 *  - G of Eq. ApoVote (kappa-scaled) is enclosed over the box in FP32
 *    interval arithmetic with the operations of pair_G and an FP32 sine
 *    enclosure (or_sinf at the ends, a 2^-20 margin, extrema wherever they
 *    may lie);
 *  - d^Ax is the FP32 point evaluation, at the box centre rounded to FP32,
 *    of or_stereo_e's operations: the transverse quantities with or_sinf,
 *    or_cosf and or_atan2f, then the (z0, tanl) part (sin and cos of the
 *    small correction by the degree-11/12 polynomials);
 *  - the vote is the interval test of or_pair_vote in FP32, each result
 *    widened by |x| 2^-23 + 2^-149 (at least one FP32 ulp), with the
 *    tolerance band widened by `slack` + 2^-24 R, a bound on |e32 - e64|
 *    (the transverse quantities are of size R and carry FP32 rounding
 *    2^-24 relative; measured |e32 - e64| <= 6.2e-9 R + 1e-9 m over the
 *    search range); axial hits take e = +-d (no slack: it is exact);
 *  - the FP32 evaluation of d^Ax is used only inside the domain where that
 *    bound holds (R <= 2048 m, |Phi - Phi^Ax| <= 1, a positive
 *    discriminant, a finite result); outside it the pair votes.
 * Every FP32 interval contains the matching FP64 one: the inputs are rounded
 * outward, the operations are inclusion-monotone, an FP32 outward rounding
 * moves an end at least half an FP32 ulp past the exact value (more than
 * FP64's two ulps), and the sine margin 2^-20 covers or_sinf's error and the
 * FP64 enclosure's 2^-50.  With |e32 - e64| <= slack + 2^-24 R, an FP32
 * level votes for every pair an FP64 level votes for.
 * ---------------------------------------------------------------------- */
static const double R32_MAX = 2048.0;

/* pi/2 = P1 + P2 + P3 (+ 2e-15): P1 and P2 carry 11 significant bits, so
 * k P1 and k P2 are exact for |k| < 2^13 */
#define PIO2F_1 0x1.92p+0f
#define PIO2F_2 0x1.fb4p-12f
#define PIO2F_3 0x1.4442d2p-24f
#define TWO_OVER_PI_F 0x1.45f306p-1f
#define PI_F 0x1.921fb6p+1f          /* pi rounded to nearest (above) */
#define PIO2_F 0x1.921fb6p+0f        /* pi/2 rounded to nearest (above) */
#define TWO_PI_F 0x1.921fb6p+2f
#define INV_TWO_PI_F 0x1.45f306p-3f
#define PIO6_F 0x1.0c1524p-1f
#define SQRT3_F 0x1.bb67aep+0f
#define TAN_PI12_F 0x1.126146p-2f
#define SIN_MARGIN_F 0x1p-20f        /* > 4x the error of or_sinf / or_cosf for |x| <= 64 */
#define EXT_FUZZ_F 0x1p-12f          /* extremum-membership slack (in turns) */

/* the FP32 numbers next to x: largest <= x, smallest >= x */
float or_rd32(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}
float or_ru32(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}
float or_wdn32(float x) { return x - fmaf(fabsf(x), 0x1p-23f, 0x1p-149f); }
float or_wup32(float x) { return x + fmaf(fabsf(x), 0x1p-23f, 0x1p-149f); }

typedef struct { float lo, hi; } ivf;
static ivf ivf_add(ivf a, ivf b) { ivf r = {or_wdn32(a.lo + b.lo), or_wup32(a.hi + b.hi)}; return r; }
static ivf ivf_sub(ivf a, ivf b) { ivf r = {or_wdn32(a.lo - b.hi), or_wup32(a.hi - b.lo)}; return r; }
static ivf ivf_mul(ivf a, ivf b) {
  float p1 = a.lo * b.lo, p2 = a.lo * b.hi, p3 = a.hi * b.lo, p4 = a.hi * b.hi;
  ivf r = {or_wdn32(fminf(fminf(p1, p2), fminf(p3, p4))), or_wup32(fmaxf(fmaxf(p1, p2), fmaxf(p3, p4)))};
  return r;
}
static ivf ivf_sqr(ivf a) {
  float l2 = a.lo * a.lo, h2 = a.hi * a.hi;
  ivf r;
  if (a.lo <= 0.0f && a.hi >= 0.0f) { r.lo = 0.0f; r.hi = or_wup32(fmaxf(l2, h2)); }
  else { r.lo = or_wdn32(fminf(l2, h2)); r.hi = or_wup32(fmaxf(l2, h2)); }
  return r;
}
static ivf ivf_twice(ivf a) { ivf r = {2.0f * a.lo, 2.0f * a.hi}; return r; }

/* sin and cos on |x| <= 1: Taylor series to degree 11 and 12 (the first
 * omitted terms are below 2e-10), Horner's rule with fused multiply-adds */
float or_sinf1(float x) {
  float z = x * x;
  float p = 1.0f / 39916800.0f;            /* 1/11! */
  p = fmaf(p, z, -1.0f / 362880.0f);       /* 1/9! */
  p = fmaf(p, z, 1.0f / 5040.0f);          /* 1/7! */
  p = fmaf(p, z, -1.0f / 120.0f);          /* 1/5! */
  p = fmaf(p, z, 1.0f / 6.0f);             /* 1/3! */
  return fmaf(-(x * z), p, x);
}
float or_cosf1(float x) {
  float z = x * x;
  float q = 1.0f / 479001600.0f;           /* 1/12! */
  q = fmaf(q, z, -1.0f / 3628800.0f);      /* 1/10! */
  q = fmaf(q, z, 1.0f / 40320.0f);         /* 1/8! */
  q = fmaf(q, z, -1.0f / 720.0f);          /* 1/6! */
  q = fmaf(q, z, 1.0f / 24.0f);            /* 1/4! */
  q = fmaf(q, z, -0.5f);                   /* 1/2! */
  return fmaf(z, q, 1.0f);
}

/* sin and cos of any argument with |x| <= 64: reduction by pi/2 (the
 * three-part constant above, in FP32), then the polynomials on |r| <= pi/4 */
static float reduce_f(float x, int *q) {
  float k = rintf(x * TWO_OVER_PI_F);
  float r = ((x - k * PIO2F_1) - k * PIO2F_2) - k * PIO2F_3;
  *q = (int)k & 3;
  return r;
}
float or_sinf(float x) {
  int q;
  float r = reduce_f(x, &q);
  float v = (q & 1) ? or_cosf1(r) : or_sinf1(r);
  return (q & 2) ? -v : v;
}
float or_cosf(float x) {
  int q;
  float r = reduce_f(x, &q);
  float v = (q & 1) ? or_sinf1(r) : or_cosf1(r);
  return ((q + 1) & 2) ? -v : v;
}

/* atan on |u| <= tan(pi/12): Taylor series to degree 13 (first omitted term
 * below 3e-10) */
static float atan_f(float u) {
  float z = u * u;
  float p = 1.0f / 13.0f;
  p = fmaf(p, z, -1.0f / 11.0f);
  p = fmaf(p, z, 1.0f / 9.0f);
  p = fmaf(p, z, -1.0f / 7.0f);
  p = fmaf(p, z, 1.0f / 5.0f);
  p = fmaf(p, z, -1.0f / 3.0f);
  return fmaf(u * z, p, u);
}
/* angle of (x, y) in [-pi, pi], the octant reduction of or_atan2 in FP32 */
float or_atan2f(float y, float x) {
  float ax = fabsf(x), ay = fabsf(y);
  if (ax == 0.0f && ay == 0.0f) return 0.0f;
  int swap = ay > ax;
  float t = swap ? ax / ay : ay / ax;
  float a;
  if (t > TAN_PI12_F) a = PIO6_F + atan_f((t * SQRT3_F - 1.0f) / (t + SQRT3_F));
  else a = atan_f(t);
  if (swap) a = PIO2_F - a;
  if (x < 0.0f) a = PI_F - a;
  if (y < 0.0f) a = -a;
  return a;
}

/* FP32 enclosure of sin over [a, b] (as or_sin_encl) */
void or_sin_encl32(float a, float b, float *lo, float *hi) {
  if (b - a >= TWO_PI_F) { *lo = -1.0f; *hi = 1.0f; return; }
  float va = or_sinf(a), vb = or_sinf(b);
  float l = fminf(va, vb) - SIN_MARGIN_F, h = fmaxf(va, vb) + SIN_MARGIN_F;
  if (floorf((b - PIO2_F) * INV_TWO_PI_F + EXT_FUZZ_F) >= ceilf((a - PIO2_F) * INV_TWO_PI_F - EXT_FUZZ_F)) h = 1.0f;
  if (floorf((b + PIO2_F) * INV_TWO_PI_F + EXT_FUZZ_F) >= ceilf((a + PIO2_F) * INV_TWO_PI_F - EXT_FUZZ_F)) l = -1.0f;
  *lo = fmaxf(l, -1.0f);
  *hi = fminf(h, 1.0f);
}

/* d^Ax at the point c for drift sign s, in FP32 as defined above.
 * Returns 1 and writes e32 = sgn(kappa) d^Ax, or 0 outside the FP32 domain
 * (then the caller votes).  dbg (nullable, 24 floats): as or_stereo_e. */
int32_t or_stereo_e32(const or_prep *h, const double c[5], int32_t s, float *e, float *dbg) {
  float cf[5];
  for (int j = 0; j < 5; j++) cf[j] = (float)c[j];   /* the centre, rounded to nearest */
  float kap = cf[2], sig = 1.0f;
  if (kap < 0.0f) sig = -1.0f;
  if (kap == 0.0f) { kap = 0x1p-30f; sig = 1.0f; }
  const float kp = sig * kap, d0p = sig * cf[0];
  const float sp0 = sig * or_sinf(cf[1]), cp0 = or_cosf(cf[1]);
  const float R = 1.0f / kp;
  if (!(R <= R32_MAX)) return 0;
  const float Rd = R + d0p;
  const float xc = -(Rd * sp0), yc = Rd * cp0;
  const float py = sig * (float)h->py, cps = sig * (float)h->cphis, sps = (float)h->sphis;
  const float Dx = (float)h->px - xc, Dy = py - yc;
  const float RAx = sqrtf(Dx * Dx + Dy * Dy);
  const float cAx = Dx * sps - Dy * cps;
  const float sAx = Dx * cps + Dy * sps;
  const float sinA = sAx / RAx, cosA = cAx / RAx;
  const float dphi = or_atan2f(Dx * cp0 + Dy * sp0, Dx * sp0 - Dy * cp0);
  const float sArc = R * dphi;
  const float c2 = cosA * cosA - sinA * sinA, s2 = 2.0f * sinA * cosA;
  const float twoRAx2 = 2.0f * (RAx * RAx), RpRAx = R + RAx;
  const float z0 = cf[3], lam = cf[4], tt = (float)h->tant;
  const float dS = (float)s * (float)h->d;
  /* the (z0, tanl) part, in the order of or_stereo_e */
  float zA = z0 + lam * sArc;
  float Phi1 = -(zA * sinA + (lam * dS) * cosA) / RAx;
  float Phi2n = (lam * R) * zA - ((lam * zA) * (R - 2.0f * dS)) * c2
              + (zA * zA + dS * (RAx + (lam * lam) * (RpRAx - dS))) * s2;
  float Phi2 = Phi2n / twoRAx2;
  float t2 = tt * tt;
  float eps = Phi1 * tt + Phi2 * t2;
  if (!(fabsf(eps) <= 1.0f)) return 0;
  float se = or_sinf1(eps), ce = or_cosf1(eps);
  float sinP = sinA * ce + cosA * se, cosP = cosA * ce - sinA * se;
  float u = sqrtf(((1.0f + ((2.0f * lam) * sinP) * tt) + (lam * lam) * t2) + (cosP * cosP) * t2);
  float delta = dS / u;
  float sperp = R * (dphi + eps);
  float zS = (z0 + lam * sperp) - (delta * cosP) * tt;
  float ctau = zS * cAx - (lam * delta) * sAx;
  float a1 = zS * tt, a2 = (lam * delta) * tt;
  float Q = ((2.0f * ctau) * tt + a1 * a1) + a2 * a2;
  float A = R + delta;
  float disc = A * A - Q;
  if (!(disc > 0.0f)) return 0;
  float dhat = delta - Q / (A + sqrtf(disc));
  if (dbg) {
    float v[24] = {R, xc, yc, Dx, Dy, RAx, cAx, sAx, sinA, cosA, dphi,
                   zA, Phi1, Phi2, eps, sinP, cosP, u, delta, sperp, zS, ctau, Q, dhat};
    memcpy(dbg, v, sizeof v);
  }
  *e = sig * dhat;
  return isfinite(*e) ? 1 : 0;
}

/* G of Eq. ApoVote (kappa-scaled) over the box, in FP32 intervals with the
 * operations of pair_G */
static ivf pair_G32(const or_prep *h, const or_box *b) {
  ivf K = {or_rd32(b->lo[2]), or_ru32(b->hi[2])}, Dd = {or_rd32(b->lo[0]), or_ru32(b->hi[0])};
  ivf Fi = {or_rd32(b->lo[1]), or_ru32(b->hi[1])};
  ivf P = {or_rd32(h->phip), or_ru32(h->phip)};
  ivf Ar = {or_wdn32(Fi.lo - P.hi), or_wup32(Fi.hi - P.lo)};
  ivf S;
  or_sin_encl32(Ar.lo, Ar.hi, &S.lo, &S.hi);
  ivf r = {or_rd32(h->r), or_ru32(h->r)};
  ivf rS = ivf_mul(S, r);
  ivf D2 = ivf_sqr(Dd);
  ivf T0 = ivf_add(D2, (ivf){or_rd32(h->r2lo), or_ru32(h->r2hi)});
  ivf T = {0.5f * T0.lo, 0.5f * T0.hi};
  ivf KT = ivf_mul(K, T);
  ivf KD1 = ivf_add(ivf_mul(K, Dd), (ivf){1.0f, 1.0f});
  return ivf_add(ivf_add(KT, ivf_mul(KD1, rS)), Dd);
}

void or_pair_G32(const or_prep *h, const or_box *b, float *lo, float *hi) {
  ivf G = pair_G32(h, b);
  *lo = G.lo;
  *hi = G.hi;
}

/* the vote of one (box, hit) at an FP32 level; dbg (nullable, 8 floats):
 * G lo/hi, H+ lo/hi, H- lo/hi, e+, e- */
int32_t or_pair_vote32(const or_prep *h, const or_box *b, double slack, float *dbg) {
  if (!h->valid) return 0;
  const ivf G = pair_G32(h, b);
  const ivf K = {or_rd32(b->lo[2]), or_ru32(b->hi[2])};
  int32_t vote = 0;
  if (dbg) { dbg[0] = G.lo; dbg[1] = G.hi; for (int j = 2; j < 8; j++) dbg[j] = NAN; }
  if (h->axial) {
    /* e = sgn(kappa) (+-d) exactly: its FP32 interval needs no slack */
    const double kc = 0.5 * (b->lo[2] + b->hi[2]);
    const float sig = (float)kc < 0.0f ? -1.0f : 1.0f;
    const float blo = or_ru32(h->band);
    for (int32_t si = 0; si < 2; si++) {
      const double e = (double)sig * (si == 0 ? h->d : -h->d);
      ivf E = {or_wdn32(or_rd32(e) - blo), or_wup32(or_ru32(e) + blo)};
      ivf H = ivf_sub(ivf_twice(G), ivf_add(ivf_twice(E), ivf_mul(K, ivf_sqr(E))));
      if (dbg) { dbg[2 + 2 * si] = H.lo; dbg[3 + 2 * si] = H.hi; dbg[6 + si] = (float)e; }
      if (H.lo <= 0.0f && 0.0f <= H.hi) vote = 1;
    }
    return vote;
  }
  double c[5];
  for (int j = 0; j < 5; j++) c[j] = 0.5 * (b->lo[j] + b->hi[j]);
  float dbg24[24];
  for (int32_t si = 0; si < 2; si++) {
    float e;
    if (!or_stereo_e32(h, c, si == 0 ? 1 : -1, &e, dbg24)) { vote = 1; continue; }
    /* the band widened by slack + 2^-24 R (R = dbg24[0], the centre's radius) */
    const float bs = or_wup32(or_wup32(or_ru32(h->band) + or_ru32(slack)) + dbg24[0] * 0x1p-24f);
    ivf E = {or_wdn32(e - bs), or_wup32(e + bs)};
    ivf H = ivf_sub(ivf_twice(G), ivf_add(ivf_twice(E), ivf_mul(K, ivf_sqr(E))));
    if (dbg) { dbg[2 + 2 * si] = H.lo; dbg[3 + 2 * si] = H.hi; dbg[6 + si] = e; }
    if (H.lo <= 0.0f && 0.0f <= H.hi) vote = 1;
  }
  return vote;
}

/* ------------------------------------------------------------------------
 * one accumulator level: votes of all active valid hits for every box
 * ---------------------------------------------------------------------- */
static int64_t prod5(const int32_t m[5]) {
  int64_t p = 1;
  for (int j = 0; j < 5; j++) p *= m[j];
  return p;
}

static void vote_prepped(const or_prep *pr, const uint8_t *use, int32_t n_hits,
                         const or_box *parents, int32_t n_parents, const int32_t split[5],
                         int32_t prec, double slack, int32_t fwd, double disk, double xr, double yr,
                         uint16_t *votes, int32_t n_threads) {
  int64_t nc = prod5(split), nb = (int64_t)n_parents * nc;
#ifdef _OPENMP
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nt)
#endif
  for (int64_t b = 0; b < nb; b++) {
    or_box box;
    or_box_child(&parents[b / nc], split, b % nc, &box);
    int32_t v = 0;
    if ((disk > 0.0 && !or_disk(&box, xr, yr, disk)) || (fwd == 2 && !or_behind(&box, xr, yr))) {
      votes[b] = 0;
      continue;
    }
    for (int32_t i = 0; i < n_hits; i++) {
      if (!use[i] || (fwd == 1 && !or_forward(&pr[i], &box))) continue;
      v += prec == OR_FP32 ? or_pair_vote32(&pr[i], &box, slack, NULL)
         : prec == OR_IV   ? or_pair_vote_iv(&pr[i], &box)
                           : or_pair_vote_x(&pr[i], &box, prec == OR_FP64X, NULL);
    }
    votes[b] = (uint16_t)v;
  }
  (void)n_threads;
}

void or_vote_level(const or_hit *hits, int32_t n_hits, const uint8_t *active,
                   const or_box *parents, int32_t n_parents, const int32_t split[5],
                   uint16_t *votes, int32_t n_threads) {
  or_vote_level_prec(hits, n_hits, active, parents, n_parents, split, OR_FP64, 0.0, votes, n_threads);
}

void or_vote_level_prec(const or_hit *hits, int32_t n_hits, const uint8_t *active,
                        const or_box *parents, int32_t n_parents, const int32_t split[5],
                        int32_t prec, double slack, uint16_t *votes, int32_t n_threads) {
  or_vote_level_ex(hits, n_hits, active, parents, n_parents, split, prec, slack, 0, 0.0, 0.0, 0.0, votes,
                   n_threads);
}

void or_vote_level_ex(const or_hit *hits, int32_t n_hits, const uint8_t *active,
                      const or_box *parents, int32_t n_parents, const int32_t split[5],
                      int32_t prec, double slack, int32_t forward, double xr, double yr,
                      double disk, uint16_t *votes, int32_t n_threads) {
  or_prep *pr = (or_prep *)calloc((size_t)(n_hits > 0 ? n_hits : 1), sizeof *pr);
  uint8_t *use = (uint8_t *)calloc((size_t)(n_hits > 0 ? n_hits : 1), 1);
  for (int32_t i = 0; i < n_hits; i++)
    use[i] = (uint8_t)(or_prep_hit_ref(&hits[i], xr, yr, &pr[i]) && (!active || active[i]));
  vote_prepped(pr, use, n_hits, parents, n_parents, split, prec, slack, forward, disk, xr, yr, votes, n_threads);
  free(pr);
  free(use);
}

/* ------------------------------------------------------------------------
 * selection of the max-vote boxes: full sort by (votes desc, index asc)
 * ---------------------------------------------------------------------- */
typedef struct { uint16_t v; int64_t idx; } vi_pair;

static int cmp_vi(const void *a, const void *b) {
  const vi_pair *x = (const vi_pair *)a, *y = (const vi_pair *)b;
  if (x->v != y->v) return x->v > y->v ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

int32_t or_topk(const uint16_t *votes, int64_t n_boxes, int32_t k, int64_t *out_index,
                uint16_t *out_votes) {
  if (n_boxes <= 0 || k <= 0) return 0;
  vi_pair *a = (vi_pair *)malloc((size_t)n_boxes * sizeof *a);
  for (int64_t b = 0; b < n_boxes; b++) { a[b].v = votes[b]; a[b].idx = b; }
  qsort(a, (size_t)n_boxes, sizeof *a, cmp_vi);
  int32_t kk = (int64_t)k < n_boxes ? k : (int32_t)n_boxes;
  for (int32_t i = 0; i < kk; i++) { out_index[i] = a[i].idx; out_votes[i] = a[i].v; }
  free(a);
  return kk;
}

/* ------------------------------------------------------------------------
 * estimate from the selected max-vote cells (Sec. 3.3): the mean of their
 * centres (phi0 taken relative to the first cell's centre, in (-pi, pi]) and
 * half the extent of their union as the error.  Sums run over the level's
 * boxes in index order by pairwise summation on a zero-padded power-of-two
 * array (cells that are not maximal contribute zero).
 * ---------------------------------------------------------------------- */
static double pairwise_sum(double *a, int64_t p2) {
  for (int64_t n = p2; n > 1; n >>= 1)
    for (int64_t i = 0; i < n / 2; i++) a[i] = a[2 * i] + a[2 * i + 1];
  return a[0];
}

int32_t or_estimate(const or_box *parents, int32_t n_parents, const int32_t split[5],
                    const uint16_t *votes, uint16_t vmax, double p[5], double err[5]) {
  double ulo[5], uhi[5];
  return or_estimate_ex(parents, n_parents, split, votes, vmax, p, err, ulo, uhi);
}

static int32_t estimate_masked(const or_box *parents, int32_t n_parents, const int32_t split[5],
                               const uint16_t *votes, uint16_t vmax, const uint8_t *mask, double p[5],
                               double err[5], double ulo[5], double uhi[5]);

int32_t or_estimate_ex(const or_box *parents, int32_t n_parents, const int32_t split[5],
                       const uint16_t *votes, uint16_t vmax, double p[5], double err[5],
                       double ulo[5], double uhi[5]) {
  return estimate_masked(parents, n_parents, split, votes, vmax, NULL, p, err, ulo, uhi);
}

/* the estimate over the max-vote boxes with mask[b] != 0 (mask NULL: all) */
static int32_t estimate_masked(const or_box *parents, int32_t n_parents, const int32_t split[5],
                               const uint16_t *votes, uint16_t vmax, const uint8_t *mask, double p[5],
                               double err[5], double ulo[5], double uhi[5]) {
  int64_t nc = prod5(split), nb = (int64_t)n_parents * nc, p2 = 1;
  while (p2 < nb) p2 <<= 1;
  double *acc[5];
  for (int j = 0; j < 5; j++) acc[j] = (double *)calloc((size_t)p2, sizeof(double));
  double lo_min[5], hi_max[5], c0 = 0.0;
  for (int j = 0; j < 5; j++) { lo_min[j] = INFINITY; hi_max[j] = -INFINITY; }
  int32_t count = 0;
  for (int64_t b = 0; b < nb; b++) {
    if (votes[b] != vmax || (mask && !mask[b])) continue;
    or_box box;
    or_box_child(&parents[b / nc], split, b % nc, &box);
    if (count == 0) c0 = 0.5 * (box.lo[1] + box.hi[1]);
    for (int j = 0; j < 5; j++) {
      double c = 0.5 * (box.lo[j] + box.hi[j]), lo = box.lo[j], hi = box.hi[j];
      if (j == 1) {
        double dv = c - c0, shift = 0.0;
        if (dv > PI_RN) shift = -TWO_PI_RN;
        else if (dv <= -PI_RN) shift = TWO_PI_RN;
        acc[j][b] = dv + shift;
        lo = lo + shift;
        hi = hi + shift;
      } else {
        acc[j][b] = c;
      }
      lo_min[j] = fmin(lo_min[j], lo);
      hi_max[j] = fmax(hi_max[j], hi);
    }
    count++;
  }
  for (int j = 0; j < 5; j++) {
    double S = pairwise_sum(acc[j], p2);
    if (count == 0) { p[j] = NAN; err[j] = NAN; continue; }
    if (j == 1) {
      double v = c0 + S / (double)count;
      if (v < 0.0) v += TWO_PI_RN;
      if (v >= TWO_PI_RN) v -= TWO_PI_RN;
      p[j] = v;
    } else {
      p[j] = S / (double)count;
    }
    err[j] = 0.5 * (hi_max[j] - lo_min[j]);
  }
  for (int j = 0; j < 5; j++) { ulo[j] = lo_min[j]; uhi[j] = hi_max[j]; }
  for (int j = 0; j < 5; j++) free(acc[j]);
  return count;
}

/* ------------------------------------------------------------------------
 * the search for one event (Sec. 3.3): coarse vote, refinement, estimate,
 * hit finding with the box estimate +- scale x error; repeated on the hits
 * not yet assigned for several helices.
 *
 * OR_TOPK: each level keeps the first top_k boxes by (votes desc, index asc)
 * and splits each by `split`.
 *
 * OR_WINDOW: each level is one regular grid over a window box.  Level 0's
 * window is the search range.  After a level, the estimate comes from ALL
 * its max-vote boxes of one phi0 run (never truncated within it: Sec. 3.3
 * computes the values and errors from every selected max cell; phi_run
 * below keeps to one track), and the next window from every box of the run
 * within wdrop votes of the maximum (noise hits can lift a few boxes by a
 * vote or two above the track's own): the union of those boxes (phi0
 * relative to the first max-vote box's centre, as in the estimate) widened
 * by one of the level's bins on each side (kappa and tanl clipped to the
 * range; d0 and z0 too while the reference point is the origin; a phi0
 * window of a full turn or more becomes the range's).  After level
 * move_level the reference point moves, as the paper does for its second and
 * third steps, to the measurement point closest to the recovered circle
 * (the active hit point with the smallest |G| at the estimate, the lowest
 * index on ties): the 32 corners of those boxes are taken to the new
 * reference point (or_frame_shift; phi0 within half a turn of the first
 * max-vote box's first corner) and the next window is their hull widened so
 * that it spans all but one bin at each end of the next grid (kappa and tanl
 * clipped).  With hitsel, as the paper does after each iteration, a level
 * votes only with the hits that vote for the previous level's hit-finding
 * box (estimate +- hitfind_scale x error, in that level's frame); every hit
 * of the pass stays a candidate at each selection and at the hit finding.
 * With `forward`, the levels about the origin (up to move_level, or all
 * when the reference point never moves, or does not find a hit) apply the
 * forward-hit test to their votes, selections and the hit finding; the
 * levels about a moved reference point apply the direction test or_behind
 * to every box instead.  With disk > 0 every level applies the disk
 * condition (or_disk) in its frame.  The helix's p is
 * the last estimate taken back to the origin; its err and the hit finding
 * stay in the last level's frame.
 * Parity of the driver: the per-level truth checks and the recovery rates
 * (A22 tolerances) are pinned on generated events; there is no paper number.
 * ---------------------------------------------------------------------- */
static uint16_t level_max(const uint16_t *votes, int64_t nb, int64_t *first) {
  uint16_t vmax = 0;
  int64_t f = 0;
  for (int64_t b = 0; b < nb; b++)
    if (votes[b] > vmax) { vmax = votes[b]; f = b; }
  *first = f;
  return vmax;
}

static void hit_finding(const or_prep *pr, uint8_t *act, int32_t n_hits, const or_box *E, int32_t fwd,
                        int32_t exact, int32_t *assigned, int32_t k, int32_t *na) {
  for (int32_t i = 0; i < n_hits; i++) {
    if (!act[i]) continue;
    if (fwd && !or_forward(&pr[i], E)) continue;
    if (or_pair_vote_x(&pr[i], E, exact, NULL)) {
      act[i] = 0;
      if (assigned) assigned[i] = k;
      (*na)++;
    }
  }
}

static int32_t find_topk(const or_hit *hits, int32_t n_hits, const or_sched *sc, or_helix *out,
                         int32_t max_out, int32_t *assigned, or_trace *trace, int32_t n_threads,
                         or_prep *pr, uint8_t *act) {
  int64_t nb0 = prod5(sc->bins), nbr = (int64_t)sc->top_k * prod5(sc->split);
  int64_t nbmax = nb0 > nbr ? nb0 : nbr;
  uint16_t *votes = (uint16_t *)malloc((size_t)nbmax * sizeof(uint16_t));
  int32_t kmax = sc->top_k;
  or_box *par = (or_box *)malloc((size_t)(kmax > 1 ? kmax : 1) * sizeof(or_box));
  or_box *nxt = (or_box *)malloc((size_t)(kmax > 1 ? kmax : 1) * sizeof(or_box));
  int64_t *tidx = (int64_t *)malloc((size_t)(kmax > 1 ? kmax : 1) * sizeof(int64_t));
  uint16_t *tv = (uint16_t *)malloc((size_t)(kmax > 1 ? kmax : 1) * sizeof(uint16_t));
  int32_t nh = 0;
  (void)hits;
  for (int32_t pass = 0; pass < sc->n_helix_max && nh < max_out; pass++) {
    int32_t n_par = 1, split[5];
    par[0] = sc->range;
    memcpy(split, sc->bins, sizeof split);
    uint16_t vmax = 0;
    int32_t stop = 0;
    for (int32_t lev = 0; lev <= sc->n_refine; lev++) {
      vote_prepped(pr, act, n_hits, par, n_par, split, sc->prec[lev], sc->fp32_slack, sc->forward, sc->disk,
                   0.0, 0.0, votes, n_threads);
      int64_t nb = (int64_t)n_par * prod5(split);
      int32_t k = or_topk(votes, nb, sc->top_k, tidx, tv);
      vmax = k > 0 ? tv[0] : 0;
      if (trace && pass < OR_MAX_PASSES && lev < OR_MAX_LEVELS) {
        trace->n_passes = pass + 1;
        trace->vmax[pass][lev] = vmax;
        int32_t na = 0;
        for (int64_t b = 0; b < nb; b++) na += votes[b] == vmax;
        trace->n_argmax[pass][lev] = na;
        for (int32_t i = 0; i < k && i < OR_MAX_K; i++) {
          trace->selected_index[pass][lev][i] = tidx[i];
          or_box_child(&par[tidx[i] / prod5(split)], split, tidx[i] % prod5(split),
                       &trace->selected[pass][lev][i]);
        }
      }
      if (lev == 0 && vmax < sc->v_min) { stop = 1; break; }   /* too few votes for a helix */
      if (lev == sc->n_refine) break;
      /* the selected boxes become the parents of the next level */
      int64_t nc = prod5(split);
      for (int32_t i = 0; i < k; i++) or_box_child(&par[tidx[i] / nc], split, tidx[i] % nc, &nxt[i]);
      for (int32_t i = 0; i < k; i++) par[i] = nxt[i];
      n_par = k;
      memcpy(split, sc->split, sizeof split);
    }
    if (stop) break;
    or_helix hx;
    memset(&hx, 0, sizeof hx);
    hx.n_argmax = or_estimate(par, n_par, split, votes, vmax, hx.p, hx.err);
    hx.votes = vmax;
    /* hit finding: every still-active hit voting for estimate +- scale x error */
    or_box E;
    for (int j = 0; j < 5; j++) {
      double w = sc->hitfind_scale * hx.err[j];
      E.lo[j] = hx.p[j] - w;
      E.hi[j] = hx.p[j] + w;
    }
    int32_t na = 0;
    hit_finding(pr, act, n_hits, &E, sc->forward, sc->prec[sc->n_refine] == OR_FP64X, assigned, nh, &na);
    hx.n_assigned = na;
    out[nh++] = hx;
    if (na == 0) break;
  }
  free(votes); free(par); free(nxt); free(tidx); free(tv);
  return nh;
}

/* corner c (bit j: upper end of dimension j) of box b */
static void box_corner(const or_box *b, int c, double x[5]) {
  for (int j = 0; j < 5; j++) x[j] = ((c >> j) & 1) ? b->hi[j] : b->lo[j];
}

/* One track at a time: at the coarse levels every helix of an event ties at
 * the maximum, and their max-vote boxes together would give a meaningless
 * estimate.  The estimate and the next window therefore use the max-vote
 * boxes (and the boxes within wdrop of the maximum) whose phi0 bin lies in
 * the contiguous run of phi0 bins holding max-vote boxes that contains the
 * first max-vote box's bin (circular when the grid spans a full turn; every
 * bin when the run covers them all or the grid has more than RUN_MAX_BINS
 * phi0 bins).  A single helix's max-vote boxes form one such run. */
#define RUN_MAX_BINS 1024

static void phi_run(const or_box *grid, const int32_t m[5], const uint16_t *votes, int64_t nb, uint16_t vmax,
                    int64_t first, int32_t *ra, int32_t *rb) {
  int32_t m1 = m[1];
  *ra = -1;
  *rb = -1;
  if (m1 > RUN_MAX_BINS) return;
  uint8_t occ[RUN_MAX_BINS];
  memset(occ, 0, sizeof occ);
  int64_t s1 = (int64_t)m[2] * m[3] * m[4];
  for (int64_t b = 0; b < nb; b++)
    if (votes[b] == vmax) occ[(b / s1) % m1] = 1;
  int32_t kf = (int32_t)((first / s1) % m1);
  int32_t circ = grid->hi[1] - grid->lo[1] >= TWO_PI_RN;
  int32_t a = kf, e = kf, n = 1;
  while (n < m1) {
    int32_t k = e + 1;
    if (k == m1) { if (!circ) break; k = 0; }
    if (!occ[k]) break;
    e = k;
    n++;
  }
  while (n < m1) {
    int32_t k = a - 1;
    if (k < 0) { if (!circ) break; k = m1 - 1; }
    if (!occ[k]) break;
    a = k;
    n++;
  }
  if (n == m1) return;
  *ra = a;
  *rb = e;
}

static int32_t in_run(int64_t b, const int32_t m[5], int32_t ra, int32_t rb) {
  if (ra < 0) return 1;
  int32_t k = (int32_t)((b / ((int64_t)m[2] * m[3] * m[4])) % m[1]);
  return ra <= rb ? (k >= ra && k <= rb) : (k >= ra || k <= rb);
}

static int32_t find_window(const or_hit *hits, int32_t n_hits, const or_sched *sc, or_helix *out,
                           int32_t max_out, int32_t *assigned, or_trace *trace, int32_t n_threads,
                           or_prep *pr, uint8_t *act) {
  int64_t nbmax = prod5(sc->bins);
  for (int32_t l = 1; l <= sc->n_refine; l++)
    if (prod5(sc->lbins[l]) > nbmax) nbmax = prod5(sc->lbins[l]);
  uint16_t *votes = (uint16_t *)malloc((size_t)nbmax * sizeof(uint16_t));
  uint8_t *mask = (uint8_t *)malloc((size_t)nbmax);
  uint8_t *sel = (uint8_t *)calloc((size_t)(n_hits > 0 ? n_hits : 1), 1);
  int32_t nh = 0;
  for (int32_t pass = 0; pass < sc->n_helix_max && nh < max_out; pass++) {
    /* every pass starts about the origin, with every active hit voting */
    double ref[2] = {0.0, 0.0};
    int32_t moved = 0;
    for (int32_t i = 0; i < n_hits; i++) {
      if (act[i]) or_prep_hit_ref(&hits[i], 0.0, 0.0, &pr[i]);
      sel[i] = act[i];
    }
    or_box grid = sc->range;
    int32_t m[5];
    memcpy(m, sc->bins, sizeof m);
    uint16_t vmax = 0;
    int32_t stop = 0, count = 0;
    double p[5], err[5], ulo[5], uhi[5];
    for (int32_t lev = 0; lev <= sc->n_refine; lev++) {
      /* about the origin the hits lie ahead; about a moved reference point
       * the origin lies behind */
      int32_t fwd = !sc->forward ? 0 : (moved ? 2 : 1);
      vote_prepped(pr, sel, n_hits, &grid, 1, m, sc->prec[lev], sc->fp32_slack, fwd, sc->disk, ref[0], ref[1],
                   votes, n_threads);
      int64_t nb = prod5(m), first;
      vmax = level_max(votes, nb, &first);
      int32_t ra, rb;
      phi_run(&grid, m, votes, nb, vmax, first, &ra, &rb);
      for (int64_t b = 0; b < nb; b++) mask[b] = (uint8_t)in_run(b, m, ra, rb);
      count = estimate_masked(&grid, 1, m, votes, vmax, mask, p, err, ulo, uhi);
      if (trace && pass < OR_MAX_PASSES && lev < OR_MAX_LEVELS) {
        trace->n_passes = pass + 1;
        trace->vmax[pass][lev] = vmax;
        trace->n_argmax[pass][lev] = count;
        trace->grid[pass][lev] = grid;
        trace->ref[pass][lev][0] = ref[0];
        trace->ref[pass][lev][1] = ref[1];
        trace->selected_index[pass][lev][0] = first;
        or_box_child(&grid, m, first, &trace->selected[pass][lev][0]);
      }
      if (lev == 0 && vmax < sc->v_min) { stop = 1; break; }
      if (lev == sc->n_refine) break;
      const int32_t *mn = sc->lbins[lev + 1];
      const uint16_t vlo = vmax > sc->wdrop ? (uint16_t)(vmax - sc->wdrop) : 0;
      if (sc->hitsel) {
        /* the hits voting for this level's hit-finding box vote at the next */
        or_box E;
        for (int j = 0; j < 5; j++) {
          double w = sc->hitfind_scale * err[j];
          E.lo[j] = p[j] - w;
          E.hi[j] = p[j] + w;
        }
        for (int32_t i = 0; i < n_hits; i++)
          sel[i] = (uint8_t)(act[i] && (fwd != 1 || or_forward(&pr[i], &E)) &&
                             or_pair_vote_x(&pr[i], &E, sc->prec[lev] == OR_FP64X, NULL));
      }
      or_box nx;
      int32_t did_move = 0;
      if (lev == sc->move_level) {
        /* the measurement point closest to the recovered circle */
        int32_t ib = -1;
        double gb = 0.0;
        for (int32_t i = 0; i < n_hits; i++) {
          if (!act[i]) continue;
          double g = fabs(or_point_G(&pr[i], p));
          if (ib < 0 || g < gb) { ib = i; gb = g; }
        }
        if (ib >= 0) {
          double dx = pr[ib].px, dy = pr[ib].py;
          double hl[5], hh[5], cref = 0.0;
          for (int j = 0; j < 5; j++) { hl[j] = INFINITY; hh[j] = -INFINITY; }
          {
            or_box fb;
            double x[5], q[5];
            or_box_child(&grid, m, first, &fb);
            box_corner(&fb, 0, x);
            or_frame_shift(x, dx, dy, q);
            cref = q[1];
          }
          for (int64_t b = 0; b < nb; b++) {
            if (votes[b] < vlo || !mask[b]) continue;
            or_box box;
            or_box_child(&grid, m, b, &box);
            for (int c = 0; c < 32; c++) {
              double x[5], q[5];
              box_corner(&box, c, x);
              or_frame_shift(x, dx, dy, q);
              double dv = q[1] - cref;
              if (dv > PI_RN) q[1] -= TWO_PI_RN;
              else if (dv <= -PI_RN) q[1] += TWO_PI_RN;
              for (int j = 0; j < 5; j++) { hl[j] = fmin(hl[j], q[j]); hh[j] = fmax(hh[j], q[j]); }
            }
          }
          for (int j = 0; j < 5; j++) {
            double bin = (hh[j] - hl[j]) / (double)(mn[j] > 2 ? mn[j] - 2 : 1);
            nx.lo[j] = hl[j] - bin;
            nx.hi[j] = hh[j] + bin;
          }
          ref[0] = ref[0] + dx;
          ref[1] = ref[1] + dy;
          moved = 1;
          did_move = 1;
          for (int32_t i = 0; i < n_hits; i++)
            if (act[i]) or_prep_hit_ref(&hits[i], ref[0], ref[1], &pr[i]);
        }
      }
      if (!did_move) {
        /* union of the boxes within wdrop of the maximum (phi0 relative to
         * the first max-vote box's centre) */
        double c0, wl[5], wh[5];
        or_box fb;
        or_box_child(&grid, m, first, &fb);
        c0 = 0.5 * (fb.lo[1] + fb.hi[1]);
        for (int j = 0; j < 5; j++) { wl[j] = INFINITY; wh[j] = -INFINITY; }
        for (int64_t b = 0; b < nb; b++) {
          if (votes[b] < vlo || !mask[b]) continue;
          or_box box;
          or_box_child(&grid, m, b, &box);
          for (int j = 0; j < 5; j++) {
            double lo = box.lo[j], hi = box.hi[j];
            if (j == 1) {
              double dv = 0.5 * (lo + hi) - c0, shift = 0.0;
              if (dv > PI_RN) shift = -TWO_PI_RN;
              else if (dv <= -PI_RN) shift = TWO_PI_RN;
              lo = lo + shift;
              hi = hi + shift;
            }
            wl[j] = fmin(wl[j], lo);
            wh[j] = fmax(wh[j], hi);
          }
        }
        for (int j = 0; j < 5; j++) {
          double w = (grid.hi[j] - grid.lo[j]) / (double)m[j];
          nx.lo[j] = wl[j] - w;
          nx.hi[j] = wh[j] + w;
        }
        if (!moved) {
          for (int j = 0; j < 5; j += 3) {
            nx.lo[j] = fmax(nx.lo[j], sc->range.lo[j]);
            nx.hi[j] = fmin(nx.hi[j], sc->range.hi[j]);
          }
        }
      }
      for (int j = 2; j < 5; j += 2) {
        nx.lo[j] = fmax(nx.lo[j], sc->range.lo[j]);
        nx.hi[j] = fmin(nx.hi[j], sc->range.hi[j]);
      }
      if (nx.hi[1] - nx.lo[1] >= TWO_PI_RN) { nx.lo[1] = sc->range.lo[1]; nx.hi[1] = sc->range.hi[1]; }
      grid = nx;
      memcpy(m, mn, sizeof m);
    }
    if (stop) break;
    or_helix hx;
    memset(&hx, 0, sizeof hx);
    hx.n_argmax = count;
    hx.votes = vmax;
    or_box E;
    for (int j = 0; j < 5; j++) {
      double w = sc->hitfind_scale * err[j];
      E.lo[j] = p[j] - w;
      E.hi[j] = p[j] + w;
    }
    int32_t fwd = sc->forward && !moved;
    int32_t na = 0;
    hit_finding(pr, act, n_hits, &E, fwd, sc->prec[sc->n_refine] == OR_FP64X, assigned, nh, &na);
    if (moved) or_frame_shift(p, -ref[0], -ref[1], hx.p);
    else memcpy(hx.p, p, sizeof hx.p);
    for (int j = 0; j < 5; j++) hx.err[j] = err[j];
    hx.ref[0] = ref[0];
    hx.ref[1] = ref[1];
    hx.n_assigned = na;
    out[nh++] = hx;
    if (na == 0) break;
  }
  free(votes);
  free(mask);
  free(sel);
  return nh;
}

int32_t or_find_helices(const or_hit *hits, int32_t n_hits, const or_sched *sc,
                        or_helix *out, int32_t max_out, int32_t *assigned,
                        or_trace *trace, int32_t n_threads) {
  int32_t nh1 = n_hits > 0 ? n_hits : 1;
  or_prep *pr = (or_prep *)calloc((size_t)nh1, sizeof *pr);
  uint8_t *act = (uint8_t *)calloc((size_t)nh1, 1);
  for (int32_t i = 0; i < n_hits; i++) {
    act[i] = (uint8_t)or_prep_hit(&hits[i], &pr[i]);
    if (assigned) assigned[i] = -1;
  }
  if (trace) memset(trace, 0, sizeof *trace);
  int32_t nh = sc->mode == OR_WINDOW
                   ? find_window(hits, n_hits, sc, out, max_out, assigned, trace, n_threads, pr, act)
                   : find_topk(hits, n_hits, sc, out, max_out, assigned, trace, n_threads, pr, act);
  free(pr);
  free(act);
  return nh;
}
