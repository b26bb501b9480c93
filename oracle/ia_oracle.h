/*
 * ia_oracle.h -- plain FP64 CPU oracle of the interval-arithmetic helix vote.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (libia, the HIP kernels) shares no code with it and never calls it.
 *
 * It follows "GPU-accelerated Interval Arithmetic to solve the Apollonius
 * Problem applied to a Stereo Drift Chamber" (da Silva, Lebrun, Angelique,
 * Del Buono):
 *   - the helix model, Eqs. HelixEq_a-d (Sec. 2.2), in perigee form;
 *   - the stereo wire and the virtual drift distance d^Ax, Appendix A
 *     (Eqs. wirePar, normudi, EQSinter, defdiAX_b, ApproxPhi);
 *   - the interval vote predicate, Eq. ApoVote (Sec. 3.1), with d^Ax taken
 *     at the middle of the voxel (Sec. 3.1, last paragraph);
 *   - the iterative max-cell refinement, the estimate from the selected
 *     voxels and the hit finding (Sec. 3.3).
 * and, for levels of a mixed-precision schedule marked OR_FP32, the FP32
 * vote or_pair_vote32 (a definition of this implementation, not the paper's).
 * Units: m, rad, 1/m.  Box dimension order: d0, phi0, kappa, z0, tanl.
 */
#ifndef IA_ORACLE_H
#define IA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double x0, y0, z0, x1, y1, z1, drift, band; } or_hit;
typedef struct { double lo[5], hi[5]; } or_box;

/* per-hit constants (Eqs. wirePar_a,b and EQSinter_d,e with z_ref = 0) */
typedef struct {
  int32_t valid, axial;
  double px, py;        /* wire point at z = 0 */
  double tant;          /* tan(tau) >= 0 */
  double sphis, cphis;  /* sin, cos of the wire projection angle phi_s */
  double r, phip;       /* polar form of (px, py); (r, phip) define the hit point */
  double r2lo, r2hi;    /* outward enclosure of r*r */
  double d, band;       /* drift radius and tolerance half-width */
} or_prep;

#define OR_MAX_LEVELS 8
/* per-level arithmetic: FP64 with the second-order Phi of Eq. ApproxPhi,
 * FP32 (see the source), FP64 with the exact Phi of Eq. CSAXtoPHI_a, or the
 * sound enclosure of d^Ax over the whole box (OR_IV) */
enum { OR_FP64 = 0, OR_FP32 = 1, OR_FP64X = 2, OR_IV = 3 };
#define OR_PHI_ITERS 3   /* fixed-point steps of Eq. CSAXtoPHI_a at OR_FP64X */
#define OR_IV_ITERS 6    /* interval fixed-point steps of Eq. CSAXtoPHI_a at OR_IV */
enum { OR_TOPK = 0, OR_WINDOW = 1 };

typedef struct {
  or_box range; int32_t bins[5];          /* level-0 regular grid */
  int32_t n_refine, top_k, split[5];      /* refinement schedule */
  int32_t v_min, n_helix_max;             /* multi-helix stop rules */
  double hitfind_scale;                   /* half-width of the hit-finding box in errors */
  int32_t prec[OR_MAX_LEVELS];            /* OR_FP64 or OR_FP32 per level */
  double fp32_slack;                      /* band widening at FP32 levels (m) */
  int32_t mode;                           /* OR_TOPK: top_k boxes split by split;
                                             OR_WINDOW: one window box per level */
  int32_t forward;                        /* forward-hit test at the levels in the
                                             origin's frame */
  int32_t move_level;                     /* OR_WINDOW: the reference point moves after
                                             this level (-1: never) */
  int32_t wdrop;                          /* OR_WINDOW: the next window covers the boxes
                                             with votes >= max - wdrop */
  int32_t hitsel;                         /* OR_WINDOW: a level votes with the hits that
                                             voted for the previous level's hit-finding box */
  int32_t lbins[OR_MAX_LEVELS][5];        /* OR_WINDOW: grid of level l >= 1 over its window */
  double disk;                            /* Eq. ApoVoteDisk: boxes whose circles all miss the
                                             disk of this radius about the origin (m) get no
                                             votes; 0: off */
} or_sched;

typedef struct {
  double p[5], err[5];   /* p about the origin; err: half extent of the max-vote
                            boxes, in the frame of the reference point ref */
  double ref[2];         /* reference point of the last level (0, 0 without a move) */
  int32_t votes, n_assigned, n_argmax, pad;
} or_helix;

#define OR_MAX_K 64
#define OR_MAX_PASSES 16
typedef struct {
  int32_t n_passes;
  int32_t vmax[OR_MAX_PASSES][OR_MAX_LEVELS];
  int32_t n_argmax[OR_MAX_PASSES][OR_MAX_LEVELS];
  or_box selected[OR_MAX_PASSES][OR_MAX_LEVELS][OR_MAX_K];
  int64_t selected_index[OR_MAX_PASSES][OR_MAX_LEVELS][OR_MAX_K];
  or_box grid[OR_MAX_PASSES][OR_MAX_LEVELS];   /* OR_WINDOW: the box each level splits */
  double ref[OR_MAX_PASSES][OR_MAX_LEVELS][2]; /* reference point of each level */
} or_trace;

/* elementary functions written for the oracle (Cody-Waite + Taylor) */
double or_sin(double x);
double or_cos(double x);
double or_atan2(double y, double x);
/* outward widening of a round-to-nearest result */
double or_wdn(double x);
double or_wup(double x);
/* interval enclosure of sin over [a, b] */
void or_sin_encl(double a, double b, double *lo, double *hi);
/* interval product (4-product rule) and square, for the tests */
void or_imul(double alo, double ahi, double blo, double bhi, double *lo, double *hi);
void or_isqr(double alo, double ahi, double *lo, double *hi);

int32_t or_prep_hit(const or_hit *h, or_prep *out);
/* the same with the hit point taken about the reference point (xr, yr):
 * px, py are the wire point at z = 0 less (xr, yr), r and phip its polar form */
int32_t or_prep_hit_ref(const or_hit *h, double xr, double yr, or_prep *out);
void or_box_child(const or_box *parent, const int32_t split[5], int64_t child, or_box *out);

/* d^Ax at the point c for drift sign s (+1 / -1).  Returns 1 and writes
 * e = sgn(kappa) d^Ax (the signed-kappa frame), or 0 when the square root of
 * Eq. defdiAX_b has a negative argument.  dbg (nullable, 24 doubles) receives
 * intermediates: see the source. */
int32_t or_stereo_e(const or_prep *h, const double c[5], int32_t s, double *e, double *dbg);
/* the same with exact = 1: Phi from Eq. CSAXtoPHI_a (OR_PHI_ITERS fixed-point
 * steps from ApproxPhi) instead of ApproxPhi */
int32_t or_stereo_e_x(const or_prep *h, const double c[5], int32_t s, int32_t exact, double *e, double *dbg);

/* Eq. ApoVote for one (box, hit): returns 1 when zero lies in the enclosure for
 * either drift sign.  dbg (nullable, 8 doubles): G lo/hi, H+ lo/hi, H- lo/hi,
 * e+, e-. */
int32_t or_pair_vote(const or_prep *h, const or_box *b, double *dbg);
/* the same with d^Ax from or_stereo_e_x(.., exact, ..) */
int32_t or_pair_vote_x(const or_prep *h, const or_box *b, int32_t exact, double *dbg);
/* IV levels: an enclosure of e = sgn(kappa) d^Ax over the whole box for drift
 * sign s (1), or 0 when none (kappa of both signs, a bound that fails); and
 * the vote with it */
int32_t or_stereo_encl(const or_prep *h, const or_box *b, int32_t s, double *lo, double *hi);
int32_t or_pair_vote_iv(const or_prep *h, const or_box *b);

/* Forward-hit test: 1 when the hit point lies ahead of the point of closest
 * approach (x cos phi0 + y sin phi0 > 0) for some phi0 of the box, 0 when it
 * lies behind for every phi0 of the box.  A hit at the reference point is
 * ahead. */
int32_t or_forward(const or_prep *h, const or_box *b);

/* perigee parameters p about a reference point -> q about that point moved
 * by (dx, dy); valid for kappa = 0 (straight lines) */
void or_frame_shift(const double p[5], double dx, double dy, double q[5]);

/* kappa-scaled residual G (Eq. ApoVote divided by 2 R) of the hit point at
 * the parameter point p: its magnitude is the distance of the hit point from
 * the circle to first order */
double or_point_G(const or_prep *h, const double p[5]);

/* FP32 levels (see the source for the definition): outward and nearest
 * FP64 -> FP32 conversions, FP32 widening, sin/cos on |x| <= 1, d^Ax in
 * FP32 (returns 0 outside the FP32 domain), and the vote of one (box, hit)
 * in FP32 with the band widened by slack. */
float or_rd32(double x);
float or_ru32(double x);
float or_wdn32(float x);
float or_wup32(float x);
float or_sinf1(float x);
float or_cosf1(float x);
int32_t or_stereo_e32(const or_prep *h, const double c[5], int32_t s, float *e, float *dbg);
/* FP32 sin, cos (|x| <= 64), atan2, the FP32 sine enclosure and G of
 * Eq. ApoVote over a box in FP32 intervals */
float or_sinf(float x);
float or_cosf(float x);
float or_atan2f(float y, float x);
void or_sin_encl32(float a, float b, float *lo, float *hi);
void or_pair_G32(const or_prep *h, const or_box *b, float *lo, float *hi);
int32_t or_pair_vote32(const or_prep *h, const or_box *b, double slack, float *dbg);

/* votes[parent * prod(split) + child] for every child box of every parent.
 * active (nullable) masks hits. */
void or_vote_level(const or_hit *hits, int32_t n_hits, const uint8_t *active,
                   const or_box *parents, int32_t n_parents, const int32_t split[5],
                   uint16_t *votes, int32_t n_threads);
/* the same at precision prec (OR_FP64 or OR_FP32, band widening slack) */
void or_vote_level_prec(const or_hit *hits, int32_t n_hits, const uint8_t *active,
                        const or_box *parents, int32_t n_parents, const int32_t split[5],
                        int32_t prec, double slack, uint16_t *votes, int32_t n_threads);

/* the same with the forward-hit test (forward = 1) or the direction test
 * or_behind (forward = 2), the hits taken about the reference point (xr, yr),
 * and the disk test of Eq. ApoVoteDisk (disk > 0) */
void or_vote_level_ex(const or_hit *hits, int32_t n_hits, const uint8_t *active,
                      const or_box *parents, int32_t n_parents, const int32_t split[5],
                      int32_t prec, double slack, int32_t forward, double xr, double yr,
                      double disk, uint16_t *votes, int32_t n_threads);

/* Eq. ApoVoteDisk for one box in the frame of the reference point (xr, yr):
 * 1 when some circle of the box passes within `disk` of the origin */
int32_t or_disk(const or_box *b, double xr, double yr, double disk);

/* Direction test about a moved reference point (xr, yr): 1 when for some
 * phi0 of the box the origin lies behind the point of closest approach
 * (the track comes from the origin), 0 when it lies ahead for every phi0.
 * The origin at the reference point counts as behind. */
int32_t or_behind(const or_box *b, double xr, double yr);

/* the first k boxes by (votes desc, index asc); returns k actually taken */
int32_t or_topk(const uint16_t *votes, int64_t n_boxes, int32_t k,
                int64_t *out_index, uint16_t *out_votes);

/* estimate from the max-vote boxes of a level (Sec. 3.3) */
int32_t or_estimate(const or_box *parents, int32_t n_parents, const int32_t split[5],
                    const uint16_t *votes, uint16_t vmax, double p[5], double err[5]);
/* the same, also writing the union [ulo, uhi] of the max-vote boxes (phi0
 * taken relative to the first one's centre, as for p) */
int32_t or_estimate_ex(const or_box *parents, int32_t n_parents, const int32_t split[5],
                       const uint16_t *votes, uint16_t vmax, double p[5], double err[5],
                       double ulo[5], double uhi[5]);

/* the whole search for one event; returns the number of helices written.
 * assigned (nullable, n_hits) receives the helix index of each hit or -1. */
int32_t or_find_helices(const or_hit *hits, int32_t n_hits, const or_sched *sched,
                        or_helix *out, int32_t max_out, int32_t *assigned,
                        or_trace *trace, int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
