// Host-side check harness: the vote arithmetic of libia (the same
// __host__ __device__ functions the HIP kernels run), compiled for the CPU
// and driven by a loop with the kernels' structure -- the (triple, hit)
// classification and per-triple bounds, the pruning threshold, then the
// per-box stereo term of the pairs left undecided.
// Used only by the tests, to compare the device arithmetic with the oracle
// on many events without a GPU.
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../paper_2401_04576_amd/csrc/ia_kernels.hpp"

using namespace ia;

static bool make_shape(const int32_t m[5], int64_t n_parents, Shape* sh) {
  int64_t nc = 1;
  for (int j = 0; j < 5; ++j) {
    if (m[j] < 1) return false;
    sh->m[j] = static_cast<uint32_t>(m[j]);
    nc *= m[j];
  }
  sh->nc = static_cast<uint32_t>(nc);
  sh->m34 = sh->m[3] * sh->m[4];
  sh->m012 = sh->m[0] * sh->m[1] * sh->m[2];
  sh->m12 = sh->m[1] * sh->m[2];
  sh->n_boxes = static_cast<uint32_t>(nc * n_parents);
  sh->n_parents = static_cast<uint32_t>(n_parents);
  return true;
}

extern "C" {

// votes of the boxes of a level at precision f32 (0: FP64, 1: FP32 with
// band widening slack), following the library's structure: classes of every
// (triple, hit) pair (with the exclusion / inclusion proofs when `filter`),
// per-triple bounds tlb (class-1 pairs) and tn2 (class-2 pairs), then the
// per-box evaluation of class-2 pairs.  With prune_k > 0 only triples whose
// upper bound reaches T (the prune_k-th largest lower bound over boxes) are
// evaluated, and with `ties` those whose upper bound is exactly T only up to
// the tie cut; the boxes of the others keep their lower bound.
// stats: [0] stereo (triple, hit) pairs, [1] class 0, [2] stereo (box, hit)
// evaluations, [3] of those that voted, [4] evaluated pairs voting in every
// box of their triple, [5] class 1, [6] triples evaluated, [7] T,
// [8] (parent, hit) pairs the parent-level test excluded (with parent_filter),
// [9] stereo pairs the first stage decided, or left with one drift sign,
// from the parent's ranges of d^Ax
int32_t hc_vote_level(const double* hits, int32_t n_hits, const double* parents, int32_t n_parents,
                      const int32_t split[5], int32_t filter, int32_t f32, double slack, int32_t prune_k,
                      int32_t ties, int32_t parent_filter, uint16_t* votes, int64_t* stats) {
  const float slack32 = ru32(slack);
  Shape sh;
  if (!make_shape(split, n_parents, &sh)) return 1;
  std::vector<HitRec> rec(n_hits > 0 ? n_hits : 1);
  for (int32_t i = 0; i < n_hits; ++i) {
    bool bad;
    prep_one(hits + 8 * i, true, &rec[i], &bad);
  }
  const BoxD* P = reinterpret_cast<const BoxD*>(parents);
  const int64_t n_triples = int64_t(n_parents) * sh.m012;
  // parent-level exclusion per (parent, hit)
  std::vector<uint8_t> pmay(size_t(n_parents) * size_t(n_hits > 0 ? n_hits : 1), 1);
  std::vector<ParentE> pe(pmay.size());
  int64_t n_pexcl = 0;
  // (the library runs no class proofs at FP32 levels)
  if (parent_filter && filter && !f32) {
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : n_pexcl)
    for (int32_t p = 0; p < n_parents; ++p)
      for (int32_t i = 0; i < n_hits; ++i) {
        const bool may = f32 ? parent_may_vote<true>(P[p], sh.m, rec[i], slack32)
                             : parent_may_vote<false>(P[p], sh.m, rec[i], slack32, &pe[size_t(p) * n_hits + i]);
        pmay[size_t(p) * n_hits + i] = may ? 1 : 0;
        n_pexcl += (!may && rec[i].use) ? 1 : 0;
      }
  }
  std::vector<uint8_t> cls(size_t(n_triples) * size_t(n_hits > 0 ? n_hits : 1));
  std::vector<int32_t> tlb(n_triples), tn2(n_triples);
  int64_t n_pairs = 0, n_cut = 0, n_incl = 0, n_prange = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : n_pairs, n_cut, n_incl, n_prange)
  for (int64_t t = 0; t < n_triples; ++t) {
    const uint32_t tp = static_cast<uint32_t>(t / sh.m012), tc = static_cast<uint32_t>(t % sh.m012);
    const Frame f = triple_frame(P[tp], sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
    Iv Zr, Lr;
    centre_ranges(P[tp], sh.m, &Zr, &Lr);
    const GTri gt = g_triple(f);
    int32_t a = 0, c2 = 0;
    for (int32_t i = 0; i < n_hits; ++i) {
      const HitRec& h = rec[i];
      uint8_t fl = 0;
      if (h.use && pmay[size_t(tp) * n_hits + i]) {
        // the kernels' two stages
        const ParentE* pr = (parent_filter && filter && !f32) ? &pe[size_t(tp) * n_hits + i] : nullptr;
        int c = f32 ? pair_stage1<true>(f, gt, h, Zr, Lr, filter, slack32, nullptr)
                    : pair_stage1<false>(f, gt, h, Zr, Lr, filter, slack32, nullptr, pr);
        if (pr && !h.axial) {
          const int c0 = pair_stage1<false>(f, gt, h, Zr, Lr, filter, slack32, nullptr);
          if (c0 < 0 && c != c0) ++n_prange;
        }
        if (c < 0)
          c = f32 ? pair_stage2<true>(f, h, Zr, Lr, slack32, -c, nullptr)
                  : pair_stage2<false>(f, h, Zr, Lr, slack32, -c, nullptr);
        fl = static_cast<uint8_t>(c);
        if (!h.axial) {
          ++n_pairs;
          n_cut += fl == 0;
          n_incl += fl == 1;
        }
      }
      cls[size_t(t) * n_hits + i] = fl;
      a += fl == 1;
      c2 += fl == 2;
    }
    tlb[t] = a;
    tn2[t] = c2;
  }
  int32_t T = 0;
  if (prune_k > 0) {
    std::vector<int64_t> h(n_hits + 1, 0);
    for (int64_t t = 0; t < n_triples; ++t) h[std::min(tlb[t], n_hits)] += 1;
    const int64_t k_eff = std::min<int64_t>(prune_k, int64_t(sh.n_boxes));
    int64_t cum = 0;
    for (int32_t v = n_hits; v >= 0; --v) {
      cum += h[v] * sh.m34;
      if (cum >= k_eff) { T = v; break; }
    }
  }
  // tie cut (k_threshold with ties): the triple at which the triples with
  // lower bound >= T first hold k_eff boxes, in index order
  int32_t tcut = INT32_MAX;
  if (prune_k > 0 && ties) {
    const int64_t k_eff = std::min<int64_t>(prune_k, int64_t(sh.n_boxes));
    int64_t cum = 0;
    for (int64_t t = 0; t < n_triples; ++t) {
      if (tlb[t] < T) continue;
      cum += sh.m34;
      if (cum >= k_eff) { tcut = static_cast<int32_t>(t); break; }
    }
  }
  int64_t n_evals = 0, n_yes = 0, n_full = 0, n_live = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : n_evals, n_yes, n_full, n_live)
  for (int64_t t = 0; t < n_triples; ++t) {
    const uint32_t tp = static_cast<uint32_t>(t / sh.m012), tc = static_cast<uint32_t>(t % sh.m012);
    const int64_t base = int64_t(tp) * sh.nc + int64_t(tc) * sh.m34;
    std::vector<int32_t> nv(sh.m34, tlb[t]);
    if (tn2[t] > 0 && triple_live(tlb[t], tn2[t], T, static_cast<uint32_t>(t), tcut)) {
      ++n_live;
      const Frame f = triple_frame(P[tp], sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
      const Frame32 g32 = frame32_of(f);
      const float R32 = g32.R, sig32 = g32.sig;
      const Iv32 K32 = to32(f.K);
      for (int32_t i = 0; i < n_hits; ++i) {
        if (cls[size_t(t) * n_hits + i] != 2) continue;
        const HitRec& h = rec[i];
        const Iv G = residual_G(f, h);
        const PairQ q = pair_quantities(f, h, G);
        const PairQ32 q32 = pair_q32_f32(g32, h, slack32);
        int64_t yes_here = 0;
        for (uint32_t l = 0; l < sh.m34; ++l) {
          const uint32_t k3 = l / sh.m[4], k4 = l % sh.m[4];
          double zlo, zhi, llo, lhi;
          child_edge(P[tp].lo[3], P[tp].hi[3], sh.m[3], k3, &zlo, &zhi);
          child_edge(P[tp].lo[4], P[tp].hi[4], sh.m[4], k4, &llo, &lhi);
          const double z0 = 0.5 * (zlo + zhi), lam = 0.5 * (llo + lhi);
          ++n_evals;
          bool v;
          if (f32) {
            const float z032 = static_cast<float>(z0), lam32 = static_cast<float>(lam);
            v = stereo_vote32(q32, R32, sig32, K32, z032, lam32, lam32 * R32, lam32 * lam32);
          } else {
            v = stereo_vote(q, f.R, f.sig, f.K, z0, lam, lam * f.R, lam * lam, h.tant, h.tant * h.tant, h.d, h.band);
          }
          if (v) { ++nv[l]; ++n_yes; ++yes_here; }
        }
        if (yes_here == int64_t(sh.m34)) ++n_full;
      }
    }
    for (uint32_t l = 0; l < sh.m34; ++l) votes[base + l] = static_cast<uint16_t>(nv[l]);
  }
  if (stats) {
    stats[0] = n_pairs; stats[1] = n_cut; stats[2] = n_evals; stats[3] = n_yes; stats[4] = n_full;
    stats[5] = n_incl; stats[6] = n_live; stats[7] = T; stats[8] = n_pexcl; stats[9] = n_prange;
  }
  return 0;
}

}  // extern "C"

extern "C" {

// magnitude bound of d^Ax (e_magnitude) for stereo hit `hit` over triple tc
// of parent `parent` split by `split`: returns 1 and writes M, the eps bound
// and the discriminant lower bound to out[0..2]; 0 when no bound exists;
// -1 for an axial or invalid hit
int32_t hc_e_magnitude(const double* hit, const double* parent, const int32_t split[5], uint32_t tc,
                       double* out) {
  Shape sh;
  if (!make_shape(split, 1, &sh)) return -1;
  HitRec h;
  bool bad;
  prep_one(hit, true, &h, &bad);
  if (!h.use || h.axial) return -1;
  const BoxD& P = *reinterpret_cast<const BoxD*>(parent);
  const Frame f = triple_frame(P, sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
  Iv Z, L;
  centre_ranges(P, sh.m, &Z, &L);
  const PairQ q = pair_quantities(f, h, residual_G(f, h));
  EMag em;
  if (!e_magnitude(q, f.R, h.tant, h.d, Z, L, &em)) return 0;
  out[0] = em.M;
  out[1] = em.eps;
  out[2] = em.disc_lo;
  return 1;
}

}  // extern "C"

extern "C" {

// residual_G and residual_G_outer of each (triple, hit) pair of one level:
// out[4 (t n_hits + i) ..] = G.lo, G.hi, Go.lo, Go.hi (0 for unused hits)
int32_t hc_g_pairs(const double* hits, int32_t n_hits, const double* parent, const int32_t split[5], double* out) {
  Shape sh;
  if (!make_shape(split, 1, &sh)) return 1;
  std::vector<HitRec> rec(n_hits > 0 ? n_hits : 1);
  for (int32_t i = 0; i < n_hits; ++i) {
    bool bad;
    prep_one(hits + 8 * i, true, &rec[i], &bad);
  }
  const BoxD& P = *reinterpret_cast<const BoxD*>(parent);
  for (uint32_t tc = 0; tc < sh.m012; ++tc) {
    const Frame f = triple_frame(P, sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
    const GTri g = g_triple(f);
    for (int32_t i = 0; i < n_hits; ++i) {
      double* o = out + 4 * (size_t(tc) * n_hits + i);
      if (!rec[i].use) { o[0] = o[1] = o[2] = o[3] = 0.0; continue; }
      const Iv G = residual_G(f, rec[i]), Go = residual_G_outer(f, g, rec[i]);
      o[0] = G.lo; o[1] = G.hi; o[2] = Go.lo; o[3] = Go.hi;
    }
  }
  return 0;
}

}  // extern "C"

// d^Ax at one box centre for one drift sign, in stereo_vote's operations;
// false where the discriminant is negative or the value is not finite
static bool point_e(const PairQ& q, double R, double sig, double z0, double lam, double tt, double t2, double dS,
                    double* e) {
  const double lamR = lam * R, lam2 = lam * lam;
  const double zA = z0 + lam * q.sArc, zAs = zA * q.sinA, zA2 = zA * zA, lzA = lam * zA;
  const double Phi1 = -(zAs + (lam * dS) * q.cosA) / q.RAx;
  const double Phi2n = lamR * zA - (lzA * (R - 2.0 * dS)) * q.c2 + (zA2 + dS * (q.RAx + lam2 * (q.RpRAx - dS))) * q.s2;
  const double eps = Phi1 * tt + (Phi2n / q.twoRAx2) * t2;
  double se, ce;
  sincos_p(eps, &se, &ce);
  const double sinP = q.sinA * ce + q.cosA * se, cosP = q.cosA * ce - q.sinA * se;
  const double u = sqrt(((1.0 + ((2.0 * lam) * sinP) * tt) + lam2 * t2) + (cosP * cosP) * t2);
  const double delta = dS / u;
  const double zS = (z0 + lam * (R * (q.dphi + eps))) - (delta * cosP) * tt;
  const double ld = lam * delta;
  const double ctau = zS * q.cAx - ld * q.sAx;
  const double a1 = zS * tt, a2 = ld * tt;
  const double Q = ((2.0 * ctau) * tt + a1 * a1) + a2 * a2;
  const double A = R + delta, disc = A * A - Q;
  if (!(disc >= 0.0)) return false;
  *e = sig * (delta - Q / (A + sqrt(disc)));
  return std::isfinite(*e);
}

extern "C" {

// For every (triple, stereo hit) pair of one parent's level and each drift
// sign: the FP64 and FP32 enclosures of e over the centre rectangle and the
// range of the point values at the boxes' centres.  Row of 10 per (triple,
// hit, sign): ok64, E64.lo, E64.hi, ok32, E32.lo, E32.hi, n_points, min, max,
// stereo (0 for an axial or unused hit).
int32_t hc_encl_pairs(const double* hits, int32_t n_hits, const double* parent, const int32_t split[5],
                      double* out) {
  Shape sh;
  if (!make_shape(split, 1, &sh)) return 1;
  std::vector<HitRec> rec(n_hits > 0 ? n_hits : 1);
  for (int32_t i = 0; i < n_hits; ++i) {
    bool bad;
    prep_one(hits + 8 * i, true, &rec[i], &bad);
  }
  const BoxD& P = *reinterpret_cast<const BoxD*>(parent);
  Iv Z, L;
  centre_ranges(P, sh.m, &Z, &L);
  for (uint32_t tc = 0; tc < sh.m012; ++tc) {
    const Frame f = triple_frame(P, sh.m, tc / sh.m12, (tc / sh.m[2]) % sh.m[1], tc % sh.m[2]);
    for (int32_t i = 0; i < n_hits; ++i) {
      const HitRec& h = rec[i];
      const bool stereo = h.use && !h.axial;
      const PairQ q = pair_quantities(f, h, residual_G(f, h));
      const double tt = h.tant, t2 = tt * tt;
      const EnclIn32 c = encl_in32(q, f.R, tt, t2, h.d, Z, L);
      for (int si = 0; si < 2; ++si) {
        double* o = out + 10 * ((size_t(tc) * n_hits + i) * 2 + si);
        for (int k = 0; k < 10; ++k) o[k] = 0.0;
        if (!stereo) continue;
        o[9] = 1.0;
        const double dS = si == 0 ? h.d : -h.d;
        Iv E = {0.0, 0.0}, EPS, DISC, A;
        o[0] = e_enclosure_dom(q, f.R, f.sig, tt, t2, ipt(dS), Z, L, &E, &EPS, &DISC, &A) ? 1.0 : 0.0;
        o[1] = E.lo; o[2] = E.hi;
        E = {0.0, 0.0};
        o[3] = e_enclosure32(c, si != 0, f.sig, &E, &EPS, &DISC, &A) ? 1.0 : 0.0;
        o[4] = E.lo; o[5] = E.hi;
        double n = 0.0, lo = INFINITY, hi = -INFINITY;
        for (uint32_t a = 0; a < sh.m[3]; ++a)
          for (uint32_t b = 0; b < sh.m[4]; ++b) {
            double zlo, zhi, llo, lhi, e;
            child_edge(P.lo[3], P.hi[3], sh.m[3], a, &zlo, &zhi);
            child_edge(P.lo[4], P.hi[4], sh.m[4], b, &llo, &lhi);
            if (!point_e(q, f.R, f.sig, 0.5 * (zlo + zhi), 0.5 * (llo + lhi), tt, t2, dS, &e)) continue;
            n += 1.0; lo = std::fmin(lo, e); hi = std::fmax(hi, e);
          }
        o[6] = n; o[7] = lo; o[8] = hi;
      }
    }
  }
  return 0;
}

}  // extern "C"
