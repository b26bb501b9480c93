// ia_math.hpp -- device arithmetic of the interval vote (gfx950, FP64).
//
// Outward rounding: every interval +, -, x endpoint is computed in
// round-to-nearest and moved outward by |x| 2^-52 + 2^-1074 (one fused
// multiply-add and one add), which is at least one ulp, so each enclosure
// contains the exact result.  Doubling, halving and negation are exact.
//
// sin, cos: Cody-Waite reduction by pi/2 with a three-part constant (parts of
// 33, 33 and 53 significant bits of pi/2) and Taylor polynomials of degree
// 17 (sin) and 16 (cos) on [-pi/4, pi/4], Horner with fused multiply-adds.
// atan2: octant reduction, atan t = pi/6 + atan((t sqrt3 - 1)/(t + sqrt3))
// above tan(pi/12), Taylor series of degree 29.  These are written here so
// results are reproducible independently of the device math library.
//
// The whole file must be compiled with -ffp-contract=off: only the explicit
// fma() calls may fuse.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// IA_HD: compiled for the device and, for the host-side checks, for the host
#define IA_HD __host__ __device__ __forceinline__

namespace ia {

// pi/2 = P1 + P2 + P3 (+ 1e-37): P1, P2 carry 33 significant bits
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kPio2a = 0x1.921fb544p+0;
constexpr double kPio2b = 0x1.0b4611a6p-34;
constexpr double kPio2c = 0x1.3198a2e037073p-69;
constexpr double kPi = 0x1.921fb54442d18p+1;      // below pi
constexpr double kTwoPi = 0x1.921fb54442d18p+2;   // below 2 pi
constexpr double kPio2 = 0x1.921fb54442d18p+0;    // below pi/2
constexpr double kPio2Up = 0x1.921fb54442d19p+0;  // above pi/2
constexpr double kPio6 = 0x1.0c152382d7366p-1;
constexpr double kSqrt3 = 0x1.bb67ae8584caap+0;
constexpr double kInvTwoPi = 0x1.45f306dc9c883p-3;
constexpr double kTanPi12 = 0x1.126145e9ecd56p-2;
constexpr double kSinMargin = 0x1p-50;   // > 4x the error of sin_p / cos_p
constexpr double kExtFuzz = 0x1p-40;     // extremum-membership slack

IA_HD double wdn(double x) { return x - fma(fabs(x), 0x1p-52, 0x1p-1074); }
IA_HD double wup(double x) { return x + fma(fabs(x), 0x1p-52, 0x1p-1074); }

// Horner step p z + c as one three-address fused multiply-add.  The
// compiler's two-address form (the accumulator tied to the destination)
// copies the coefficient, which stays live in a register, into the
// destination first; written as v_fma_f64 it needs no copy.  The result is
// the same correctly rounded fma.
IA_HD double horner(double p, double z, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(z), "s"(c));
  return r;
#else
  return fma(p, z, c);
#endif
}

// Square root and division forms for the per-box vote (device only).
//
// sqrt_fast: on 2^-767 <= x <= DBL_MAX the compiler's IEEE square root is a
// reciprocal-square-root start followed by two coupled Newton steps on
// (sqrt x, 1 / (2 sqrt x)) in fused multiply-adds (Markstein's scheme); its
// range scaling and its selects for 0 and infinity are identities there.
// This is that sequence without them, so the bits are the same; outside the
// range it clears *ok (the caller then takes sqrt).
// lo, hi: a narrower range the caller needs (within the one above).
IA_HD double sqrt_fast(double x, bool* ok, double lo = 0x1p-767, double hi = 0x1.fffffffffffffp+1023) {
#if defined(__HIP_DEVICE_COMPILE__)
  *ok = *ok & (x >= lo) & (x <= hi);   // no short-circuit branches
  const double g = __builtin_amdgcn_rsq(x);
  double s = x * g, h = 0.5 * g;
  const double r = fma(-h, s, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  double d = fma(-s, s, x);
  s = fma(d, h, s);
  d = fma(-s, s, x);
  return fma(d, h, s);
#else
  (void)ok;
  return sqrt(x);
#endif
}

// Division by a value that many quotients share.  The compiler's IEEE
// quotient n / d is: r = rcp(d) refined by two Newton steps, q = n r, then
// q + r (n - d q) in fused multiply-adds, wrapped in a range scaling and a
// special-case fix-up that are both identities when d lies in
// [2^-300, 2^300] and the quotient in [2^-500, 2^500] (then n is finite,
// nonzero and far from both ends of the exponent range).  recip_v gives that
// r once per divisor (NaN outside the range); div_fast finishes one quotient
// from it with the same operations, so the bits are those of n / d, and
// clears *ok when the estimate q is outside the range (which covers n = 0,
// an infinite or NaN n, and a NaN r).  On the host r is unused.
IA_HD double recip_v(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (!(d >= 0x1p-300 && d <= 0x1p300)) return __builtin_nan("");
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / d;
#endif
}

// The same reciprocal without the range check, for a divisor the caller
// keeps in [2^-300, 2^300]; with a dividend of magnitude in [2^-200, 2^200]
// the quotient lies in [2^-500, 2^500], and div_exact finishes it as n / d.
IA_HD double rcp_newton(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / d;
#endif
}

IA_HD double div_exact(double n, double d, double r) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double q = n * r;
  return fma(fma(-d, q, n), r, q);
#else
  (void)r;
  return n / d;
#endif
}

IA_HD double div_fast(double n, double d, double r, bool* ok) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double q = n * r;
  const double aq = fabs(q);
  *ok = *ok & (aq >= 0x1p-500) & (aq <= 0x1p500);
  return fma(fma(-d, q, n), r, q);
#else
  (void)r;
  (void)ok;
  return n / d;
#endif
}

IA_HD double poly_sin(double r) {
  double z = r * r;
  double p = 1.0 / 355687428096000.0;      // 1/17!
  p = horner(p, z, -1.0 / 1307674368000.0);   // 1/15!
  p = horner(p, z, 1.0 / 6227020800.0);       // 1/13!
  p = horner(p, z, -1.0 / 39916800.0);        // 1/11!
  p = horner(p, z, 1.0 / 362880.0);           // 1/9!
  p = horner(p, z, -1.0 / 5040.0);            // 1/7!
  p = horner(p, z, 1.0 / 120.0);              // 1/5!
  p = horner(p, z, -1.0 / 6.0);               // 1/3!
  return fma(r * z, p, r);
}

IA_HD double poly_cos(double r) {
  double z = r * r;
  double q = 1.0 / 20922789888000.0;       // 1/16!
  q = horner(q, z, -1.0 / 87178291200.0);     // 1/14!
  q = horner(q, z, 1.0 / 479001600.0);        // 1/12!
  q = horner(q, z, -1.0 / 3628800.0);         // 1/10!
  q = horner(q, z, 1.0 / 40320.0);            // 1/8!
  q = horner(q, z, -1.0 / 720.0);             // 1/6!
  q = horner(q, z, 1.0 / 24.0);               // 1/4!
  q = horner(q, z, -0.5);                     // 1/2!
  return fma(z, q, 1.0);
}

// x = k pi/2 + r
IA_HD double reduce_quadrant(double x, int* quad) {
  double k = rint(x * kTwoOverPi);
  double r = ((x - k * kPio2a) - k * kPio2b) - k * kPio2c;
  *quad = static_cast<int>(static_cast<int64_t>(k) & 3);
  return r;
}

IA_HD double sin_p(double x) {
  int q;
  double r = reduce_quadrant(x, &q);
  double v = (q & 1) ? poly_cos(r) : poly_sin(r);
  return (q & 2) ? -v : v;
}

IA_HD double cos_p(double x) {
  int q;
  double r = reduce_quadrant(x, &q);
  double v = (q & 1) ? poly_sin(r) : poly_cos(r);
  return ((q + 1) & 2) ? -v : v;
}

// sin and cos of the same argument with one reduction
IA_HD void sincos_p(double x, double* s, double* c) {
  int q;
  double r = reduce_quadrant(x, &q);
  double ps = poly_sin(r), pc = poly_cos(r);
  double sv = (q & 1) ? pc : ps;
  double cv = (q & 1) ? ps : pc;
  *s = (q & 2) ? -sv : sv;
  *c = ((q + 1) & 2) ? -cv : cv;
}

// below pi/4 in magnitude the reduction of sincos_p is the identity (k = 0,
// r = x exactly), so the polynomials alone give sincos_p's values bit for bit
constexpr double kPio4 = 0x1.921fb54442d18p-1;   // below pi/4

IA_HD double poly_atan(double u) {
  double z = u * u;
  double p = 1.0 / 29.0;
  p = horner(p, z, -1.0 / 27.0);
  p = horner(p, z, 1.0 / 25.0);
  p = horner(p, z, -1.0 / 23.0);
  p = horner(p, z, 1.0 / 21.0);
  p = horner(p, z, -1.0 / 19.0);
  p = horner(p, z, 1.0 / 17.0);
  p = horner(p, z, -1.0 / 15.0);
  p = horner(p, z, 1.0 / 13.0);
  p = horner(p, z, -1.0 / 11.0);
  p = horner(p, z, 1.0 / 9.0);
  p = horner(p, z, -1.0 / 7.0);
  p = horner(p, z, 1.0 / 5.0);
  p = horner(p, z, -1.0 / 3.0);
  return fma(u * z, p, u);
}

// angle of (x, y) in [-pi, pi]; 0 at the origin
IA_HD double atan2_p(double y, double x) {
  double ax = fabs(x), ay = fabs(y);
  if (ax == 0.0 && ay == 0.0) return 0.0;
  bool swap = ay > ax;
  double t = swap ? ax / ay : ay / ax;
  double a;
  if (t > kTanPi12) a = kPio6 + poly_atan((t * kSqrt3 - 1.0) / (t + kSqrt3));
  else a = poly_atan(t);
  if (swap) a = kPio2 - a;
  if (x < 0.0) a = kPi - a;
  if (y < 0.0) a = -a;
  return a;
}

struct Iv { double lo, hi; };

IA_HD Iv iadd(Iv a, Iv b) { return {wdn(a.lo + b.lo), wup(a.hi + b.hi)}; }
IA_HD Iv isub(Iv a, Iv b) { return {wdn(a.lo - b.hi), wup(a.hi - b.lo)}; }
IA_HD Iv imul(Iv a, Iv b) {
  double p1 = a.lo * b.lo, p2 = a.lo * b.hi, p3 = a.hi * b.lo, p4 = a.hi * b.hi;
  return {wdn(fmin(fmin(p1, p2), fmin(p3, p4))), wup(fmax(fmax(p1, p2), fmax(p3, p4)))};
}
// interval times a non-negative point: the 4-product rule reduces to two products
IA_HD Iv imul_pos(Iv a, double s) { return {wdn(a.lo * s), wup(a.hi * s)}; }
IA_HD Iv isqr(Iv a) {
  double l2 = a.lo * a.lo, h2 = a.hi * a.hi;
  if (a.lo <= 0.0 && a.hi >= 0.0) return {0.0, wup(fmax(l2, h2))};
  return {wdn(fmin(l2, h2)), wup(fmax(l2, h2))};
}
IA_HD Iv itwice(Iv a) { return {2.0 * a.lo, 2.0 * a.hi}; }
IA_HD Iv ipt(double x) { return {x, x}; }
IA_HD Iv ineg(Iv a) { return {-a.hi, -a.lo}; }
// a / p for a point p > 0
IA_HD Iv idivp(Iv a, double p) { return {wdn(a.lo / p), wup(a.hi / p)}; }
// a / b for b > 0: the quotient is monotone in each argument
IA_HD Iv idiv_pos(Iv a, Iv b) {
  double q1 = a.lo / b.lo, q2 = a.lo / b.hi, q3 = a.hi / b.lo, q4 = a.hi / b.hi;
  return {wdn(fmin(fmin(q1, q2), fmin(q3, q4))), wup(fmax(fmax(q1, q2), fmax(q3, q4)))};
}
// square root of [lo, hi] with hi >= 0; negative parts are clipped
IA_HD Iv isqrt(Iv a) { return {a.lo > 0.0 ? wdn(sqrt(a.lo)) : 0.0, wup(sqrt(a.hi))}; }

// interval times a point of either sign: two products
IA_HD Iv imul_pt(Iv a, double x) {
  const double p = a.lo * x, q = a.hi * x;
  return x >= 0.0 ? Iv{wdn(p), wup(q)} : Iv{wdn(q), wup(p)};
}
// a / b for b.lo > 0: the extreme quotients, chosen by the signs of a's ends
IA_HD Iv idiv_pos2(Iv a, Iv b) {
  const double lo = a.lo / (a.lo >= 0.0 ? b.hi : b.lo);
  const double hi = a.hi / (a.hi >= 0.0 ? b.lo : b.hi);
  return {wdn(lo), wup(hi)};
}

// sin and cos enclosures for intervals inside [-kSmallTrig, kSmallTrig]:
// there sin increases and cos decreases with |x|; Taylor polynomials of
// degree 13 and 14 are within 1e-14 of them, far below the 2^-40 margin
constexpr double kSmallTrig = 0.75;
constexpr double kSmallMargin = 0x1p-40;
IA_HD double sin_small(double x) {
  const double z = x * x;
  double p = 1.0 / 6227020800.0;
  p = horner(p, z, -1.0 / 39916800.0);
  p = horner(p, z, 1.0 / 362880.0);
  p = horner(p, z, -1.0 / 5040.0);
  p = horner(p, z, 1.0 / 120.0);
  p = horner(p, z, -1.0 / 6.0);
  return fma(x * z, p, x);
}
IA_HD double cos_small(double x) {
  const double z = x * x;
  double q = -1.0 / 87178291200.0;
  q = horner(q, z, 1.0 / 479001600.0);
  q = horner(q, z, -1.0 / 3628800.0);
  q = horner(q, z, 1.0 / 40320.0);
  q = horner(q, z, -1.0 / 720.0);
  q = horner(q, z, 1.0 / 24.0);
  q = horner(q, z, -0.5);
  return fma(z, q, 1.0);
}
IA_HD void sincos_encl_small(Iv x, Iv* S, Iv* C) {
  *S = {fmax(sin_small(x.lo) - kSmallMargin, -1.0), fmin(sin_small(x.hi) + kSmallMargin, 1.0)};
  const double alo = fabs(x.lo), ahi = fabs(x.hi);
  const bool has0 = x.lo <= 0.0 && x.hi >= 0.0;
  const double amin = has0 ? 0.0 : fmin(alo, ahi), amax = fmax(alo, ahi);
  *C = {cos_small(amax) - kSmallMargin, has0 ? 1.0 : fmin(cos_small(amin) + kSmallMargin, 1.0)};
}

// enclosure of sin over [a, b]
IA_HD Iv sin_encl(double a, double b) {
  if (b - a >= kTwoPi) return {-1.0, 1.0};
  double va = sin_p(a), vb = sin_p(b);
  double l = fmin(va, vb) - kSinMargin, h = fmax(va, vb) + kSinMargin;
  if (floor((b - kPio2) * kInvTwoPi + kExtFuzz) >= ceil((a - kPio2) * kInvTwoPi - kExtFuzz)) h = 1.0;
  if (floor((b + kPio2) * kInvTwoPi + kExtFuzz) >= ceil((a + kPio2) * kInvTwoPi - kExtFuzz)) l = -1.0;
  if (l < -1.0) l = -1.0;
  if (h > 1.0) h = 1.0;
  return {l, h};
}

// enclosure of cos over [a, b] as sin over [a + pi/2, b + pi/2]
IA_HD Iv cos_encl(double a, double b) { return sin_encl(wdn(a + kPio2), wup(b + kPio2Up)); }

// ---------------------------------------------------------------------------
// FP32 levels.  Outward FP32 rounding widens by |x| 2^-23 + 2^-149 (at least
// one FP32 ulp); FP64 values enter FP32 intervals rounded outward
// (rd32 / ru32) and FP32 point arithmetic rounded to nearest.
struct Iv32 { float lo, hi; };

IA_HD float next_down32(float f) {
  if (f == 0.0f) return -0x1p-149f;
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u = f > 0.0f ? u - 1u : u + 1u;
  return __builtin_bit_cast(float, u);
}
IA_HD float next_up32(float f) { return -next_down32(-f); }
// largest FP32 <= x, smallest FP32 >= x
IA_HD float rd32(double x) {
  float f = static_cast<float>(x);
  return static_cast<double>(f) > x ? next_down32(f) : f;
}
IA_HD float ru32(double x) {
  float f = static_cast<float>(x);
  return static_cast<double>(f) < x ? next_up32(f) : f;
}
IA_HD float wdn32(float x) { return x - fmaf(fabsf(x), 0x1p-23f, 0x1p-149f); }
IA_HD float wup32(float x) { return x + fmaf(fabsf(x), 0x1p-23f, 0x1p-149f); }

IA_HD Iv32 iadd32(Iv32 a, Iv32 b) { return {wdn32(a.lo + b.lo), wup32(a.hi + b.hi)}; }
IA_HD Iv32 isub32(Iv32 a, Iv32 b) { return {wdn32(a.lo - b.hi), wup32(a.hi - b.lo)}; }
IA_HD Iv32 imul32(Iv32 a, Iv32 b) {
  float p1 = a.lo * b.lo, p2 = a.lo * b.hi, p3 = a.hi * b.lo, p4 = a.hi * b.hi;
  return {wdn32(fminf(fminf(p1, p2), fminf(p3, p4))), wup32(fmaxf(fmaxf(p1, p2), fmaxf(p3, p4)))};
}
IA_HD Iv32 isqr32(Iv32 a) {
  float l2 = a.lo * a.lo, h2 = a.hi * a.hi;
  if (a.lo <= 0.0f && a.hi >= 0.0f) return {0.0f, wup32(fmaxf(l2, h2))};
  return {wdn32(fminf(l2, h2)), wup32(fmaxf(l2, h2))};
}
IA_HD Iv32 itwice32(Iv32 a) { return {2.0f * a.lo, 2.0f * a.hi}; }
IA_HD Iv32 to32(Iv a) { return {rd32(a.lo), ru32(a.hi)}; }
IA_HD Iv32 ineg32(Iv32 a) { return {-a.hi, -a.lo}; }
// FP32 interval holding the FP64 value x: x rounded to nearest is within half
// an FP32 ulp (2^-150 in the subnormal range) of x, and the widening moves
// each end by at least one ulp
IA_HD Iv32 thin32(double x) {
  const float f = static_cast<float>(x);
  return {wdn32(f), wup32(f)};
}
// FP32 interval holding the FP64 interval a (same argument per end)
IA_HD Iv32 cover32(Iv a) { return {wdn32(static_cast<float>(a.lo)), wup32(static_cast<float>(a.hi))}; }
// quotients and roots are widened by |x| 2^-21 + 2^-149 (at least four ulps),
// which holds them whether or not the device rounds them correctly
IA_HD float wdn32q(float x) { return x - fmaf(fabsf(x), 0x1p-21f, 0x1p-149f); }
IA_HD float wup32q(float x) { return x + fmaf(fabsf(x), 0x1p-21f, 0x1p-149f); }
// a / b for b.lo > 0: the extreme quotients, chosen by the signs of a's ends
IA_HD Iv32 idiv_pos32(Iv32 a, Iv32 b) {
  const float lo = a.lo / (a.lo >= 0.0f ? b.hi : b.lo);
  const float hi = a.hi / (a.hi >= 0.0f ? b.lo : b.hi);
  return {wdn32q(lo), wup32q(hi)};
}
// square root of [lo, hi] with hi >= 0; negative parts are clipped
IA_HD Iv32 isqrt32(Iv32 a) { return {a.lo > 0.0f ? wdn32q(sqrtf(a.lo)) : 0.0f, wup32q(sqrtf(a.hi))}; }

// sin and cos for |x| <= 1: Taylor polynomials of degree 11 and 12 (first
// omitted terms below 2e-10), Horner with fused multiply-adds
IA_HD float sin1_32(float x) {
  float z = x * x;
  float p = 1.0f / 39916800.0f;
  p = fmaf(p, z, -1.0f / 362880.0f);
  p = fmaf(p, z, 1.0f / 5040.0f);
  p = fmaf(p, z, -1.0f / 120.0f);
  p = fmaf(p, z, 1.0f / 6.0f);
  return fmaf(-(x * z), p, x);
}
IA_HD float cos1_32(float x) {
  float z = x * x;
  float q = 1.0f / 479001600.0f;
  q = fmaf(q, z, -1.0f / 3628800.0f);
  q = fmaf(q, z, 1.0f / 40320.0f);
  q = fmaf(q, z, -1.0f / 720.0f);
  q = fmaf(q, z, 1.0f / 24.0f);
  q = fmaf(q, z, -0.5f);
  return fmaf(z, q, 1.0f);
}

// sin and cos enclosures for FP32 intervals inside [-0.75, 0.75], where sin
// increases and cos decreases with |x|.  On that range the polynomials above
// are within 4e-12 of sin and cos and their FP32 evaluation within 2e-7 (a
// few roundings of values below 1); the margin 2^-21 (4.8e-7) covers both.
constexpr float kSmallTrig32 = 0.75f;
constexpr float kSmallMargin32 = 0x1p-21f;
IA_HD void sincos_encl_small32(Iv32 x, Iv32* S, Iv32* C) {
  *S = {fmaxf(sin1_32(x.lo) - kSmallMargin32, -1.0f), fminf(sin1_32(x.hi) + kSmallMargin32, 1.0f)};
  const float alo = fabsf(x.lo), ahi = fabsf(x.hi);
  const bool has0 = x.lo <= 0.0f && x.hi >= 0.0f;
  const float amin = has0 ? 0.0f : fminf(alo, ahi), amax = fmaxf(alo, ahi);
  *C = {cos1_32(amax) - kSmallMargin32, has0 ? 1.0f : fminf(cos1_32(amin) + kSmallMargin32, 1.0f)};
}

// FP32 levels evaluate the whole predicate in FP32: sin and cos of any
// argument with |x| <= 64 by reduction with a three-part pi/2 (11, 11 and 24
// significant bits: k P1 and k P2 exact for |k| < 2^13) and the polynomials
// above on |r| <= pi/4; atan2 by the octant reduction of atan2_p with a
// degree-13 Taylor series on |u| <= tan(pi/12); the FP32 sine enclosure with
// a 2^-20 margin (more than 4x the error of sinf32 there).
constexpr float kPio2F1 = 0x1.92p+0f;
constexpr float kPio2F2 = 0x1.fb4p-12f;
constexpr float kPio2F3 = 0x1.4442d2p-24f;
constexpr float kTwoOverPiF = 0x1.45f306p-1f;
constexpr float kPiF = 0x1.921fb6p+1f;
constexpr float kPio2F = 0x1.921fb6p+0f;
constexpr float kTwoPiF = 0x1.921fb6p+2f;
constexpr float kInvTwoPiF = 0x1.45f306p-3f;
constexpr float kPio6F = 0x1.0c1524p-1f;
constexpr float kSqrt3F = 0x1.bb67aep+0f;
constexpr float kTanPi12F = 0x1.126146p-2f;
constexpr float kSinMarginF = 0x1p-20f;
constexpr float kExtFuzzF = 0x1p-12f;

IA_HD float reduce_f32(float x, int* q) {
  const float k = rintf(x * kTwoOverPiF);
  const float r = ((x - k * kPio2F1) - k * kPio2F2) - k * kPio2F3;
  *q = static_cast<int>(k) & 3;
  return r;
}
IA_HD float sinf32(float x) {
  int q;
  const float r = reduce_f32(x, &q);
  const float v = (q & 1) ? cos1_32(r) : sin1_32(r);
  return (q & 2) ? -v : v;
}
IA_HD float cosf32(float x) {
  int q;
  const float r = reduce_f32(x, &q);
  const float v = (q & 1) ? sin1_32(r) : cos1_32(r);
  return ((q + 1) & 2) ? -v : v;
}
IA_HD float atan_f32(float u) {
  const float z = u * u;
  float p = 1.0f / 13.0f;
  p = fmaf(p, z, -1.0f / 11.0f);
  p = fmaf(p, z, 1.0f / 9.0f);
  p = fmaf(p, z, -1.0f / 7.0f);
  p = fmaf(p, z, 1.0f / 5.0f);
  p = fmaf(p, z, -1.0f / 3.0f);
  return fmaf(u * z, p, u);
}
IA_HD float atan2f32(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  if (ax == 0.0f && ay == 0.0f) return 0.0f;
  const bool swap = ay > ax;
  const float t = swap ? ax / ay : ay / ax;
  float a;
  if (t > kTanPi12F) a = kPio6F + atan_f32((t * kSqrt3F - 1.0f) / (t + kSqrt3F));
  else a = atan_f32(t);
  if (swap) a = kPio2F - a;
  if (x < 0.0f) a = kPiF - a;
  if (y < 0.0f) a = -a;
  return a;
}
IA_HD Iv32 sin_encl32(float a, float b) {
  if (b - a >= kTwoPiF) return {-1.0f, 1.0f};
  const float va = sinf32(a), vb = sinf32(b);
  float l = fminf(va, vb) - kSinMarginF, h = fmaxf(va, vb) + kSinMarginF;
  if (floorf((b - kPio2F) * kInvTwoPiF + kExtFuzzF) >= ceilf((a - kPio2F) * kInvTwoPiF - kExtFuzzF)) h = 1.0f;
  if (floorf((b + kPio2F) * kInvTwoPiF + kExtFuzzF) >= ceilf((a + kPio2F) * kInvTwoPiF - kExtFuzzF)) l = -1.0f;
  return {fmaxf(l, -1.0f), fminf(h, 1.0f)};
}

}  // namespace ia
