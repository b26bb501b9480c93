/*
 * ia.h -- C ABI of libia, the MI355X (gfx950) interval-arithmetic helix vote.
 *
 * Method: da Silva, Lebrun, Angelique, Del Buono, "GPU-accelerated Interval
 * Arithmetic to solve the Apollonius Problem applied to a Stereo Drift
 * Chamber".  Every hit -- a drift radius and the two end points of its wire
 * (Sec. 3.2) -- votes for each box of helix-parameter space whose interval
 * enclosure of the Apollonius tangency condition (Eq. ApoVote, with the
 * stereo virtual drift distance d^Ax of Eq. defdiAX_b taken at the middle of
 * the box, Sec. 3.1) contains zero, for either drift sign.  The max-vote
 * boxes are selected, subdivided and voted again level by level (Sec. 3.3).
 *
 * Parameters (SI units: m, rad, 1/m), always in this order:
 *   d0     signed distance of closest approach to the z axis
 *   phi0   direction of travel at that point, [0, 2 pi)
 *   kappa  signed curvature 1/R, > 0 for counter-clockwise seen from +z
 *   z0     z at the point of closest approach
 *   tanl   dz / ds_perp (the paper's lambda)
 * The transverse circle has centre (1/kappa + d0)(-sin phi0, cos phi0).
 *
 * Box order: a level is n_parents parent boxes each split regularly by
 * split[5]; box b = parent * prod(split) + child with the child index
 * lexicographic (d0 slowest, tanl fastest).  Child edges along a dimension
 * with range [L, U] and m parts are L + k (U - L)/m, and the last edge is U.
 * A level-0 grid is the case n_parents = 1, parent = the search range.
 * There is no call that lists a level's boxes: every kernel computes a box
 * from (parent, child index) with this formula.
 *
 * Conventions shared by every entry point:
 *  - Pointers named d_* are device memory owned by the caller; the library
 *    never frees them.  h_* and plain struct pointers are host memory, read
 *    during the call.
 *  - Work is enqueued on `stream` (a hipStream_t, passed as void *); the calls
 *    return without waiting.  One context must be used by one stream at a
 *    time: its scratch is reused by every call.
 *  - The return value reports errors the host can see (null pointers, sizes,
 *    scratch too small, HIP launch failures).  Problems found on the device
 *    (malformed hits, a vote above the bound) are recorded in the context and
 *    read with ia_ctx_status() after the stream has been synchronised.
 *    Malformed hits (non-finite values, z0 == z1, drift < 0, band < 0) never
 *    vote; they are counted, not fatal.
 *  - No entry point allocates device memory except ia_ctx_create.
 *  - Results are deterministic: integer votes and fixed reduction orders do
 *    not depend on launch shapes or on other work on the device.
 */
#ifndef IA_H
#define IA_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IA_OK = 0,
  IA_ERR_INVALID = 1,      /* bad argument */
  IA_ERR_NOMEM = 2,        /* context scratch too small for the request */
  IA_ERR_DEVICE = 3,       /* a HIP call failed */
  IA_ERR_UNSUPPORTED = 4,  /* valid request this build does not implement */
  IA_ERR_OVERFLOW = 5      /* a size does not fit the index types */
} ia_status;

/* Arithmetic of a level.  IA_FP64: d^Ax with the second-order Phi of Eq.
 * ApproxPhi (Appendix A), the paper's form.  IA_FP32: see ia_vote_level.
 * IA_FP64X: FP64 with the exact Phi, the solution of Eq. CSAXtoPHI_a by
 * three fixed-point steps from ApproxPhi; the closest approach is then
 * independent of z_ref, which stays 0.  IA_IV: the sound test -- d^Ax
 * enclosed over the whole box (every quantity of Appendix A in FP64 interval
 * arithmetic, Phi enclosed by interval fixed-point steps of Eq.
 * CSAXtoPHI_a) instead of its value at the middle of the voxel (Sec. 3.1), so
 * a box that holds a tangent helix always gets the vote.  At IA_FP64X and
 * IA_IV levels the (triple, hit) class proofs (which enclose the ApproxPhi
 * form) are off: every stereo pair is evaluated box by box. */
typedef enum { IA_FP64 = 0, IA_FP32 = 1, IA_FP64X = 2, IA_IV = 3 } ia_precision;

/* one hit: wire end points (z0 != z1), measured drift radius >= 0 and the
 * tolerance half-width added on both sides of the drift (0 = exact) */
typedef struct { double x0, y0, z0, x1, y1, z1, drift, band; } ia_hit;

typedef struct { double lo[5], hi[5]; } ia_box;

/* estimate from the max-vote boxes of a level (Sec. 3.3) */
typedef struct {
  double p[5];        /* mean of the box centres; phi0 taken relative to the
                         first max-vote box's centre in (-pi, pi], wrapped to [0, 2 pi) */
  double err[5];      /* half the extent of the union of the max-vote boxes */
  int32_t vmax;       /* the maximum vote */
  int32_t n_argmax;   /* number of boxes with vmax votes */
} ia_estimate_t;

typedef struct {
  double p[5];          /* estimate at the last level, about the origin */
  double err[5];        /* half the extent of the last level's max-vote boxes, in
                           the parameters about ref */
  double ref[2];        /* reference point of the last level ((0, 0) unless the
                           window schedule moved it) */
  int32_t votes;        /* max vote at the last level */
  int32_t n_assigned;   /* hits assigned to this helix by hit finding */
  int32_t n_argmax;     /* boxes sharing the max vote at the last level */
  int32_t status;       /* 0 */
} ia_helix;

#define IA_MAX_LEVELS 8

/* schedule modes of ia_find_helices */
enum { IA_SCHED_TOPK = 0, IA_SCHED_WINDOW = 1 };

/* the search schedule of ia_find_helices.
 *
 * IA_SCHED_TOPK: level 0 is the grid `bins` over `range`; each later level
 * splits the first top_k boxes of the previous one, by (votes desc, index
 * asc), by `split`.
 *
 * IA_SCHED_WINDOW (the paper's iterative re-gridding, Sec. 3.3 and Table 1):
 * every level is one regular grid over a window box, level 0 the grid `bins`
 * over `range`, level l >= 1 the grid lbins[l] over a window built from the
 * boxes of level l - 1 within wdrop votes of its maximum (all of them, never
 * truncated; the estimate uses the max-vote boxes alone): their union (phi0
 * relative to the first max-vote box's centre) widened by one of that
 * level's bins on each side (kappa and tanl clipped to `range`, d0 and z0 too
 * while the reference point is the origin; a phi0 window of a full turn or
 * more becomes range's).  After level move_level the reference point of the
 * parametrisation moves to the measurement point closest to the recovered
 * circle (Sec. 3.3, second and third steps): the hit point (wire at z = 0) of
 * the active hit with the smallest |G| of Eq. ApoVote's kappa-scaled form at
 * the estimate, the lowest index on ties; the next window is then the hull of
 * those boxes' 32 corners taken to the new reference point (phi0 within half
 * a turn of the first max-vote box's first corner), widened so that it spans
 * all but one bin at each end of the next grid (kappa and tanl clipped).
 * top_k and split are not used.
 *
 * forward: the paper's particles start at the origin.  About the origin a hit
 * votes for a box only if it lies ahead of the point of closest approach
 * (along the direction of travel) for some phi0 of the box (interval test on
 * cos(phi0 - phi_hit)); this removes the mirror twin (-d0, phi0 + pi, -kappa,
 * z0, -tanl) that traces the same helix backwards and otherwise ties every
 * helix.  About a moved reference point a box gets votes only if, for some
 * phi0 of it, the origin lies behind the point of closest approach.  The
 * hit-finding box and the per-level hit selection use the first test while
 * the event's reference point is the origin. */
typedef struct {
  ia_box range;           /* level-0 search range */
  int32_t bins[5];        /* level-0 grid */
  int32_t n_refine;       /* refinement levels after level 0 (< IA_MAX_LEVELS) */
  int32_t top_k;          /* IA_SCHED_TOPK: boxes kept per level, by (votes desc, index asc) */
  int32_t split[5];       /* IA_SCHED_TOPK: split of every kept box at the next level */
  int32_t v_min;          /* stop when the level-0 max vote is below this */
  int32_t n_helix_max;    /* helices searched per event (greedy, hits removed) */
  double hitfind_scale;   /* hit-finding box = estimate +- scale x error (5 in Sec. 3.3) */
  int32_t prec[IA_MAX_LEVELS];  /* arithmetic per level (ia_precision); the hit finding and
                                 * hit selection use the estimating level's with IA_FP64X,
                                 * else the FP64 mid-voxel test */
  double fp32_slack;      /* band widening at FP32 levels, m, in [0, 1e-3], to which
                           * 2^-24 R is added per box (R the radius at its centre):
                           * together they bound |e32 - e64| of d^Ax (measured at
                           * most 6.2e-9 R + 1e-9 m over the search range) */
  int32_t mode;           /* IA_SCHED_TOPK or IA_SCHED_WINDOW */
  int32_t forward;        /* 1: forward-hit test (see above), 0: off */
  int32_t move_level;     /* IA_SCHED_WINDOW: the reference point moves after this
                           * level (-1: never; else in [0, n_refine)) */
  int32_t wdrop;          /* IA_SCHED_WINDOW: windows cover the boxes with votes
                           * >= max - wdrop (>= 0) */
  int32_t hitsel;         /* IA_SCHED_WINDOW, 1: per-level hit selection (Sec. 3.3):
                           * a level votes only with the hits voting for the
                           * previous level's hit-finding box (estimate +-
                           * hitfind_scale x error, in its frame, with its
                           * forward test); every hit of the pass stays a
                           * candidate for each selection and for hit finding */
  int32_t lbins[IA_MAX_LEVELS][5];  /* IA_SCHED_WINDOW: grid of level l >= 1 */
  double disk;            /* Eq. ApoVoteDisk (Sec. 3.1), m, >= 0 (0: off): a box
                           * gets votes only if some circle of it passes within
                           * `disk` of the origin, the emission point -- the
                           * vote of a measurement at the origin with drift 0
                           * and tolerance `disk`, in each level's frame */
} ia_schedule;

typedef struct ia_ctx ia_ctx;

/* Create a context on HIP device `device` owning `scratch_bytes` of device
 * scratch, the only device allocation the library makes.  On error *out is
 * NULL.  ia_ctx_scratch_needed() gives the size a workload needs. */
ia_status ia_ctx_create(ia_ctx **out, int32_t device, size_t scratch_bytes);
void ia_ctx_destroy(ia_ctx *ctx);

/* Message of the last host-side error on this context ("" if none); with
 * ctx NULL, of this thread's last ia_vote_level_noalloc call. */
const char *ia_last_error(const ia_ctx *ctx);

/* Device-detected conditions since the last clear: flags bit 0 = malformed
 * hits seen (their number in *n_bad_hits), bit 2 = an event of
 * ia_find_helices_dev outside its declared bounds, bit 1 = a vote above the bound
 * given to ia_refine.  Synchronises the device.  Either pointer may be NULL. */
ia_status ia_ctx_status(ia_ctx *ctx, uint32_t *flags, int64_t *n_bad_hits);
ia_status ia_ctx_clear_status(ia_ctx *ctx);

/* Work counters of the vote kernel since the last ia_ctx_clear_status():
 * stereo (box, hit) evaluations performed and (triple, stereo hit) records
 * staged, at FP64 levels and at FP32 levels (pairs the pre-pass proved
 * unable to vote are in none of them).  Synchronises the device.  Any
 * pointer may be NULL. */
ia_status ia_ctx_work(ia_ctx *ctx, int64_t *stereo_box_evals, int64_t *staged_pairs,
                      int64_t *stereo_box_evals_fp32, int64_t *staged_pairs_fp32);

/* Kernel timing: while enabled, every launch of the vote kernel made through
 * this context is bracketed by HIP events on its stream.
 * ia_ctx_profile_read() synchronises the device, returns the number of
 * bracketed launches and their summed duration in milliseconds, separately
 * for FP64 and FP32 levels, and clears the record.  Creating the events is
 * the only host-side cost.  Any output pointer may be NULL. */
ia_status ia_ctx_set_profiling(ia_ctx *ctx, int32_t enable);
ia_status ia_ctx_profile_read(ia_ctx *ctx, int64_t *n_launches, double *total_ms,
                              int64_t *n_launches_fp32, double *total_ms_fp32);

/* Kernels bracketed while profiling is enabled: the vote kernel and the two
 * stages of the (triple, hit) classification run before it (the interval
 * test of Eq. ApoVote over all boxes of a triple): the first decides the
 * pairs its cheap tests can, the second runs the per-sign enclosures of
 * d^Ax on the stereo pairs left over. */
enum { IA_KERNEL_VOTE = 0, IA_KERNEL_CLASSIFY = 1, IA_KERNEL_CLASSIFY_DEFER = 2 };

/* Every bracketed launch: n_launches[2 k + p] and total_ms[2 k + p] for
 * kernel k (IA_KERNEL_*) at precision p (0 FP64 levels, 1 FP32 levels).
 * A level's vote counts once: the fallback vote of events whose staged
 * records did not fit is timed together with the record vote before it.
 * Synchronises on the recorded events and clears the record (as
 * ia_ctx_profile_read, which returns the vote kernel's entries of it).
 * Both arrays are host memory of 6 entries; IA_ERR_INVALID if either is
 * NULL. */
ia_status ia_ctx_profile_kernels(ia_ctx *ctx, int64_t n_launches[6], double total_ms[6]);

/* Counting of the classification kernel's work (off by default): while
 * enabled, the classification runs a variant that adds its work to the
 * counters ia_ctx_classify_work reads, a few per cent slower.  Results do
 * not depend on it. */
ia_status ia_ctx_set_work_counting(ia_ctx *ctx, int32_t enable);

/* Work of the two classification stages, counted while work counting was
 * enabled, since the last ia_ctx_clear_status: counts[8 p + c] at precision
 * p (0 FP64 levels, 1 FP32 levels).  First stage: c = 0 outer enclosures of
 * the residual G (Eq. ApoVote over a triple), 1 axial tests, 2 exact G for
 * axial pairs the outer one did not exclude, 3 stereo pair magnitudes,
 * 4 magnitude bounds of d^Ax (each with its exclusion test); at FP64
 * refinement levels, c = 3 and 4 leave out the stereo pairs the parent's
 * per-sign ranges of d^Ax already excluded.  Second stage: c = 5 deferred
 * pairs (each with its triple's frame, exact G and pair quantities),
 * 6 interval enclosures of d^Ax (one per drift sign left open, each with its
 * exclusion test), 7 inclusion proofs.  Only pairs of live triples are
 * counted; pairs the parent-level test excluded are not.  Synchronises the
 * device.  counts is host memory of 16 entries. */
ia_status ia_ctx_classify_work(ia_ctx *ctx, int64_t counts[16]);

/* Frame of ia_vote_level (default: forward test off, reference point at the
 * origin): with forward = 1 a hit votes only where it lies ahead of the
 * point of closest approach, with forward = 2 a box gets votes only where the
 * origin lies behind its point of closest approach (the tests described at
 * ia_schedule), and the
 * hit points are taken about the reference point (xr, yr) -- the wire point
 * at z = 0 less (xr, yr) -- so the boxes are perigee parameters about it;
 * with disk > 0 the disk condition of ia_schedule applies.  IA_ERR_INVALID
 * for a non-finite reference point or a negative or non-finite disk. */
ia_status ia_ctx_set_vote_frame(ia_ctx *ctx, int32_t forward, double xr, double yr, double disk);

/* Band widening used by ia_vote_level at IA_FP32 (default 1e-6 m; ia_find_helices
 * takes it from the schedule).  IA_ERR_INVALID outside [0, 1e-3]. */
ia_status ia_ctx_set_fp32_slack(ia_ctx *ctx, double slack);

/* Boxes per workgroup of the vote kernel: 256, 128 or 64 (the workgroup's
 * 256 lanes then split each hit chunk over 1, 2 or 4 waves), or 0 to choose
 * by level size.  Results do not depend on it. */
ia_status ia_ctx_set_vote_tile(ia_ctx *ctx, int32_t boxes_per_workgroup);

/* The (triple, hit) classification's proofs: an interval enclosure of the
 * stereo drift over every box centre sharing (d0, phi0, kappa) proves that a
 * stereo hit votes in none or in all of those boxes, and their per-box
 * evaluations are skipped.  mode -1 (the default) and 1 enable, 0 disables
 * (every stereo pair is then evaluated per box).  Results do not depend on
 * it. */
ia_status ia_ctx_set_prefilter(ia_ctx *ctx, int32_t mode);

/* Pruning in ia_find_helices: per level, each triple's votes are bounded
 * from below by its pairs proved to vote everywhere and from above by adding
 * the pairs left undecided; a triple whose upper bound is below the k-th
 * largest lower bound over boxes holds no box the selection can take, so its
 * boxes are not evaluated.  mode 0: off; 1: that threshold; 2 (default):
 * under the window schedule each level first votes the few triples with the
 * largest upper bounds (a probe), and the largest vote found there, when it
 * is above the largest lower bound, takes that bound's place in the
 * threshold (the maximum is at least both).  Selections, estimates and
 * helices do not depend on the mode; only the internal vote array of a level
 * differs (pruned boxes hold their lower bound).  IA_ERR_INVALID for another
 * mode. */
ia_status ia_ctx_set_pruning(ia_ctx *ctx, int32_t mode);

/* Parent-level exclusion in ia_find_helices (enabled by default): at each
 * refinement level, an interval enclosure over all of a parent's children
 * (their frames, pair quantities and stereo drifts) proves that a hit votes
 * for none of them, and its per-triple classification is skipped.  Results
 * do not depend on it. */
ia_status ia_ctx_set_parent_filter(ia_ctx *ctx, int32_t enable);

/* ia_find_helices launches its events in batches: every kernel of a level
 * covers all events of a batch (one event per grid row).  A batch holds as
 * many events as the scratch arena fits, at most max_events (default 65535).
 * Results do not depend on it. */
ia_status ia_ctx_set_batch(ia_ctx *ctx, int32_t max_events);

/* Scratch bytes needed by ia_find_helices for a batch of one event of at most
 * max_hits hits under `sched` (each further event of the batch needs about
 * the same again). */
size_t ia_ctx_scratch_needed(const ia_schedule *sched, int32_t max_hits);

/* One accumulator level (Eq. ApoVote over every box; Sec. 3.1).
 *   d_hits    n_hits hits (n_hits in [0, 65535])
 *   d_active  NULL or n_hits bytes; 0 excludes a hit
 *   d_parents n_parents boxes (lo <= hi in every dimension)
 *   split     host int32[5], each >= 1
 *   prec      IA_FP64; or IA_FP32: the whole predicate of each (box, hit)
 *             pair in FP32 -- G over the box in FP32 intervals, d^Ax at the
 *             box centre in FP32, the FP32 interval test with the band
 *             widened by the context's slack + 2^-24 R -- whose votes contain
 *             the IA_FP64 votes; IA_FP64X: FP64 with the exact Phi of Eq.
 *             CSAXtoPHI_a; or IA_IV: d^Ax enclosed over the whole box
 *   d_votes   n_parents * prod(split) uint16, written: number of active,
 *             well-formed hits voting for each box
 * Scratch: 112 bytes per hit, and n_parents * prod(split[0..2]) * (n_hits + 8)
 * bytes of (triple, hit) classes and per-triple bounds (IA_ERR_NOMEM when the
 * context's scratch cannot hold them); n_parents * prod(split[0..2]) * n_hits
 * below 2^31 (IA_ERR_OVERFLOW). */
ia_status ia_vote_level(ia_ctx *ctx, const ia_hit *d_hits, int32_t n_hits, const uint8_t *d_active,
                        const ia_box *d_parents, int32_t n_parents, const int32_t split[5],
                        ia_precision prec, uint16_t *d_votes, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * level as ia_vote_level, without a context.  Its scratch (hit records,
 * (triple, hit) classes, per-triple bounds, status words) is a fixed array of
 * IA_NOALLOC_SCRATCH_BYTES in the library's device code, one per device,
 * held until the process ends; the call allocates nothing and makes no
 * hipMalloc / hipFree.  Arguments as ia_vote_level; the context settings take
 * their defaults (classification proofs on, automatic vote tile, no vote
 * frame, FP32 slack 1e-6 m).
 *  - IA_ERR_NOMEM when the level needs more scratch than the array holds:
 *    n_hits x 112 bytes + n_parents x prod(split[0..2]) x (n_hits + 8) bytes
 *    + about 17 KiB must not exceed IA_NOALLOC_SCRATCH_BYTES.
 *  - Calls on one device share its array: calls that overlap on one GPU
 *    (several streams, several threads) race and must be serialised by the
 *    caller.  Each call clears what must start at zero.
 *  - Malformed hits never vote; their count is not reported (there is no
 *    context to hold it).
 *  - Host-side errors: ia_last_error(NULL) returns this thread's last
 *    message. */
#define IA_NOALLOC_SCRATCH_BYTES (64u << 20)
ia_status ia_vote_level_noalloc(const ia_hit *d_hits, int32_t n_hits, const uint8_t *d_active,
                                const ia_box *d_parents, int32_t n_parents, const int32_t split[5],
                                ia_precision prec, uint16_t *d_votes, void *stream);

/* Selection of the max-vote boxes of a level (Sec. 3.3): the first
 * min(top_k, n_boxes) boxes by (votes desc, box index asc), in that order.
 * It returns the selected boxes themselves (the next level's parents), not
 * their children: ia_vote_level splits parents itself, so children are never
 * stored.
 *   d_votes           n_boxes = n_parents * prod(split) votes, each <= vote_bound
 *   d_selected        written: the selected boxes' extents (next level's parents)
 *   d_selected_index  written: their box indices (int64)
 *   d_selected_votes  written: their votes
 * top_k in [1, 4096].  Votes above vote_bound set status bit 1 and are not
 * counted by the threshold search. */
ia_status ia_refine(ia_ctx *ctx, const ia_box *d_parents, int32_t n_parents, const int32_t split[5],
                    const uint16_t *d_votes, int32_t vote_bound, int32_t top_k, ia_box *d_selected,
                    int64_t *d_selected_index, uint16_t *d_selected_votes, void *stream);

/* Estimate from the max-vote boxes of a level (Sec. 3.3), FP64.  Sums run
 * over the level's boxes in index order by pairwise summation on a
 * zero-padded power-of-two array (non-maximal boxes add zero). */
ia_status ia_estimate(ia_ctx *ctx, const ia_box *d_parents, int32_t n_parents, const int32_t split[5],
                      const uint16_t *d_votes, ia_estimate_t *d_out, void *stream);

/* The whole search (Sec. 3.3) for n_events events.  Event e owns hits
 * [h_hit_offsets[e], h_hit_offsets[e+1]) of d_hits (host array of
 * n_events + 1 offsets, non-decreasing, each event <= 65535 hits; the
 * offsets are on the host because the call sizes the batch's per-event
 * slices from them -- ia_find_helices_dev takes them on the device).  Per
 * helix pass: vote the level-0 grid; stop if its max vote is below v_min;
 * n_refine times build the next level (IA_SCHED_WINDOW: one grid over the
 * window of the selected boxes, the reference point moved after move_level;
 * IA_SCHED_TOPK: the children of the top_k boxes) and vote it; estimate from
 * the max-vote boxes; assign every still-active hit voting for the box
 * estimate +- hitfind_scale x error; stop when none is assigned or
 * n_helix_max / max_per_event helices are found.  Helices carry no truth
 * flags: the library never sees generated truth.
 *   d_out      n_events * max_per_event helices (event-major)
 *   d_n_out    n_events counts
 *   d_assigned NULL or one int32 per hit: helix index within its event, -1 if none */
ia_status ia_find_helices(ia_ctx *ctx, const ia_hit *d_hits, const int32_t *h_hit_offsets,
                          int32_t n_events, const ia_schedule *sched, ia_helix *d_out,
                          int32_t max_per_event, int32_t *d_n_out, int32_t *d_assigned, void *stream);

/* Vote-tile autotuner: runs the search on a sample batch (as ia_find_helices,
 * writing d_out and d_n_out) once per tile size 256, 128 and 64 boxes per
 * workgroup, times the vote kernel per level size (boxes per event), and
 * keeps the fastest tile for each size; the context's automatic tile choice
 * uses that table afterwards (ia_ctx_set_vote_tile still overrides it).
 * Synchronises the stream.  Results never depend on the tile. */
ia_status ia_ctx_autotune(ia_ctx *ctx, const ia_hit *d_hits, const int32_t *h_hit_offsets, int32_t n_events,
                          const ia_schedule *sched, ia_helix *d_out, int32_t max_per_event, int32_t *d_n_out,
                          void *stream);
/* The autotuned table: writes up to max_entries (level size, tile) pairs and
 * returns the number of entries. */
int32_t ia_ctx_tuned(const ia_ctx *ctx, uint32_t *n_boxes, int32_t *tiles, int32_t max_entries);

/* The same search with the offsets on the device, for callers that capture
 * the call into a HIP graph and replay it (a persistent batch form): it
 * enqueues kernels only -- no host read of offsets, no copy, no
 * synchronisation, no allocation -- so the work depends on the host only
 * through n_events, max_hits and n_hits_total, which a replay keeps.
 *   d_off         device, n_events + 1 non-decreasing offsets into d_hits
 *   n_events      [1, 65535], all in one launch sequence (no chunking)
 *   max_hits      hits of the largest event, in [1, 65535]
 *   n_hits_total  hits addressable from d_hits (>= d_off[n_events])
 * An event with more than max_hits hits or outside [0, n_hits_total) is not
 * searched (0 helices) and sets status bit 2.  IA_ERR_NOMEM when the context
 * scratch cannot hold n_events events of max_hits hits (see
 * ia_ctx_scratch_needed).  Profiling must be off while capturing. */
ia_status ia_find_helices_dev(ia_ctx *ctx, const ia_hit *d_hits, const int32_t *d_off, int32_t n_events,
                              int32_t max_hits, int64_t n_hits_total, const ia_schedule *sched,
                              ia_helix *d_out, int32_t max_per_event, int32_t *d_n_out,
                              int32_t *d_assigned, void *stream);

/* Resident pools: continuous batching for serving, at helix-pass
 * granularity (the search of Sec. 3.3 with events arriving over time).  A
 * pool keeps `rows` event rows of up to max_hits hits each, with the whole
 * per-event search state (prepared hits, window, reference point, helices
 * found, hits assigned), resident in the context's scratch arena.  New
 * events are admitted into free rows at any time; each ia_pool_step runs one
 * helix pass -- every level of the window schedule -- over all rows still
 * searching, so events admitted at different times share the launches.  A
 * row's helices and assignments equal those of ia_find_helices for that
 * event alone (the search treats every event independently).  Only the
 * window schedule (IA_SCHED_WINDOW) is supported.  While a pool exists the
 * context's other search and vote calls return IA_ERR_INVALID (they would
 * overwrite the arena).
 *
 * ia_pool_capacity: rows of max_hits hits that fit the context's arena (0 if
 * none).  ia_pool_create: lays the pool out (every row empty) and enqueues
 * its initialisation on `stream`; IA_ERR_NOMEM if it does not fit; one pool
 * per context.  ia_pool_destroy: releases the layout (no device work). */
int32_t ia_pool_capacity(const ia_ctx *ctx, int32_t max_hits, const ia_schedule *sched, int32_t max_per_event);
ia_status ia_pool_create(ia_ctx *ctx, int32_t rows, int32_t max_hits, const ia_schedule *sched,
                         int32_t max_per_event, void *stream);
ia_status ia_pool_destroy(ia_ctx *ctx);

/* Admit n events into rows h_rows[0..n) (host, distinct, each in [0, rows)):
 * event j is hits [h_off[j], h_off[j+1]) of d_hits (device; h_off on the
 * host, non-decreasing, each event at most max_hits hits).  The hits are
 * copied into the row (d_hits may be reused once the stream has passed this
 * call) and the row restarts its search: a row still searching is abandoned.
 * n <= min(rows, 32767). */
ia_status ia_pool_admit(ia_ctx *ctx, int32_t n, const int32_t *h_rows, const ia_hit *d_hits,
                        const int32_t *h_off, void *stream);

/* One helix pass over every row still searching (enqueued on `stream`).  A
 * row finishes when its level-0 maximum is below v_min, when hit finding
 * assigns no hit, or after min(n_helix_max, max_per_event) helices. */
ia_status ia_pool_step(ia_ctx *ctx, void *stream);

/* Per-row state after the work enqueued so far: h_state[2 r] = 1 when row r
 * is not searching (finished, or never admitted), h_state[2 r + 1] = helices
 * it has written.  Synchronises the stream.  h_state: host, 2 * rows int32. */
ia_status ia_pool_poll(ia_ctx *ctx, int32_t *h_state, void *stream);

/* Copies the first n_helices helices of row `row` to h_out and the helix
 * index (-1: none) of its first n_hits hits to h_assigned (host arrays).
 * Synchronises the stream. */
ia_status ia_pool_take(ia_ctx *ctx, int32_t row, int32_t n_helices, ia_helix *h_out, int32_t n_hits,
                       int32_t *h_assigned, void *stream);

#ifdef __cplusplus
}
#endif
#endif
