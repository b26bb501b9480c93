// ia_lib.hip -- host side of libia: context, argument checks, launches.
// The C ABI is declared in include/ia.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/ia.h"
#include "ia_kernels.hpp"

using ia::BoxD;
using ia::EventState;
using ia::HitRec;
using ia::Shape;

static_assert(sizeof(ia_hit) == 64, "ia_hit layout");
static_assert(sizeof(ia_box) == sizeof(BoxD), "ia_box layout");
static_assert(sizeof(ia_helix) == sizeof(ia::HelixOut), "ia_helix layout");
static_assert(sizeof(ia_estimate_t) == sizeof(ia::EstimateOut), "ia_estimate_t layout");
static_assert(sizeof(HitRec) == 112, "HitRec layout");
static_assert(sizeof(ia::ParentE) == 40, "ParentE layout");

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kMaxHits = 65535;
constexpr int32_t kMaxTopK = ia::kMaxTopK;
constexpr int64_t kMaxLevelBoxes = (int64_t(1) << 31) - 1;
constexpr int64_t kSelChunkMin = 4096;
constexpr int32_t kSelMaxGroups = 1024;
constexpr int kOffSlots = 8;             // pinned offset-staging slots
constexpr int32_t kOffSlotInts = 65536;  // events + 1 per slot
// vote and staging workgroups per launch over the live items: 16 per resident
// slot (4 per CU on 256 CUs), so that the dispatcher, which starts a new
// workgroup as soon as one ends, balances tiles of very different record
// counts
constexpr uint32_t kVoteGroups = 16384;
// workgroups per event of the window-extent and estimate scans over the live
// tiles.  The window scan takes about kWinTotal workgroups over the batch,
// between 8 and 32 per event: in a large batch most of its workgroups do
// little more than start (8 per event run 4,096 events 23 % faster than 32),
// while a single event needs 32 to spread its tiles.  The estimate's chunk
// trees keep 32 per event busy.
constexpr int32_t kWinTotal = 32768;
constexpr int32_t kWinGroupsMin = 8, kWinGroupsMax = 32;
constexpr int32_t kEstGroups = 32;
constexpr int64_t kRecCap = 32768;       // staged records per event when the arena cannot hold all pairs
// k_estimate: 256 lanes x segments of at most 2^(kEstLevels - 1) boxes
constexpr int64_t kMaxEstimateBoxes = int64_t(ia::kWG) << (ia::kEstLevels - 1);

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// messages of ia_vote_level_noalloc (it has no context), per thread
thread_local char g_noalloc_err[512] = "";

struct Persistent {        // fixed region at the start of the arena
  uint32_t status;
  uint32_t done_counter;
  int64_t n_bad;
  // vote-kernel work counters (ia::kWorkSlots slots, summed on read)
  alignas(128) unsigned long long work[ia::kWorkSlots * ia::kWorkSlotU64];
};

}  // namespace

struct PoolState;

struct ia_ctx {
  int32_t device = 0;
  PoolState* pool = nullptr;      // a resident pool holds the arena (ia_pool_create)
  char* errbuf = nullptr;         // when set, error messages go here (no heap use)
  char* arena = nullptr;
  size_t arena_bytes = 0;
  size_t used = 0;
  std::string err;
  bool profiling = false;
  int32_t tile_override = 0;
  int32_t filter_mode = -1;       // -1: automatic, 0: off, 1: on
  int32_t prune = 2;              // ia_find_helices: skip triples that cannot reach the selection (2: with a probe)
  int32_t parent_filter = 1;      // ia_find_helices: parent-level exclusion at refinement levels
  int32_t count_work = 0;         // classification launches count their work
  int32_t max_chunk = 65535;      // events per batched launch
  float slack32 = ia::ru32(1e-6);  // band widening of ia_vote_level at FP32
  int32_t vf_forward = 0;         // ia_vote_level: forward-hit test
  double vf_xr = 0.0, vf_yr = 0.0;  // ia_vote_level: reference point
  double vf_disk = 0.0;           // ia_vote_level: disk condition radius
  // pinned staging ring for the chunk-relative hit offsets copied to the
  // device; a slot is rewritten only after its previous copy has completed
  int32_t* pinned = nullptr;
  hipEvent_t slot_done[kOffSlots] = {};
  bool slot_used[kOffSlots] = {};
  uint32_t slot_next = 0;
  struct Mark { hipEvent_t e0, e1; bool f32; uint32_t n_boxes; int32_t kind; };   // kind: IA_KERNEL_*
  std::vector<Mark> marks;
  // autotuned vote tile per level size (boxes per event), from ia_ctx_autotune
  std::vector<std::pair<uint32_t, int32_t>> tuned;
};

namespace {

ia_status fail(ia_ctx* c, ia_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c && c->errbuf) std::snprintf(c->errbuf, 512, "%s", buf);
  else if (c) c->err = buf;
  return st;
}

#define IA_HIP(c, call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail((c), IA_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

Persistent* persistent(ia_ctx* c) { return reinterpret_cast<Persistent*>(c->arena); }

void reset_bump(ia_ctx* c) { c->used = align_up(sizeof(Persistent)); }

template <typename T>
T* bump(ia_ctx* c, size_t n) {
  size_t off = align_up(c->used);
  size_t bytes = align_up(n * sizeof(T) + 1);
  if (off + bytes > c->arena_bytes) return nullptr;
  c->used = off + bytes;
  return reinterpret_cast<T*>(c->arena + off);
}

bool make_shape(const int32_t m[5], int64_t n_parents, Shape* sh) {
  int64_t nc = 1;
  for (int j = 0; j < 5; ++j) {
    if (m[j] < 1 || m[j] > (1 << 20)) return false;
    sh->m[j] = static_cast<uint32_t>(m[j]);
    nc *= m[j];
    if (nc > kMaxLevelBoxes) return false;
  }
  if (n_parents < 1 || nc * n_parents > kMaxLevelBoxes) return false;
  sh->nc = static_cast<uint32_t>(nc);
  sh->m34 = static_cast<uint32_t>(m[3]) * static_cast<uint32_t>(m[4]);
  sh->m012 = static_cast<uint32_t>(m[0]) * static_cast<uint32_t>(m[1]) * static_cast<uint32_t>(m[2]);
  sh->m12 = static_cast<uint32_t>(m[1]) * static_cast<uint32_t>(m[2]);
  sh->n_boxes = static_cast<uint32_t>(nc * n_parents);
  sh->n_parents = static_cast<uint32_t>(n_parents);
  sh->pad = 0;
  return true;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int32_t sel_groups(int64_t n_boxes, uint32_t* chunk) {
  int64_t g = (n_boxes + kSelChunkMin - 1) / kSelChunkMin;
  g = std::max<int64_t>(1, std::min<int64_t>(g, kSelMaxGroups));
  int64_t c = (n_boxes + g - 1) / g;
  c = (c + ia::kWG - 1) / ia::kWG * ia::kWG;
  *chunk = static_cast<uint32_t>(c);
  return static_cast<int32_t>((n_boxes + c - 1) / c);
}

// chunks of 256 boxes of the zero-padded power-of-two array of a level
int32_t est_parts(uint32_t n_boxes) {
  uint32_t p2 = 256;
  while (p2 < n_boxes) p2 <<= 1;
  return static_cast<int32_t>(p2 / 256);
}

// chunks per k_est_partial workgroup: enough workgroups (about 2048) to fill
// the device, at most kEstPer chunks each (n_part is a power of two)
uint32_t est_per(int32_t n_part, int32_t n_ev) {
  uint32_t per = 1;
  while (per < static_cast<uint32_t>(ia::kEstPer) && per < static_cast<uint32_t>(n_part) &&
         int64_t(n_part) * std::max(1, n_ev) / (2 * per) >= 2048)
    per <<= 1;
  return per;
}

// launches the selection of one level: histogram already in `hist`
ia_status launch_select(ia_ctx* c, const uint16_t* votes, const Shape& sh, const BoxD* parents,
                        uint32_t* hist, int32_t n_bins, int32_t top_k, int32_t* cnt, uint32_t* tmp_idx,
                        BoxD* out_boxes, int64_t* out_index, uint16_t* out_votes, EventState* ev,
                        int32_t v_min_stop, hipStream_t s) {
  uint32_t chunk;
  const int32_t g = sel_groups(sh.n_boxes, &chunk);
  hipLaunchKernelGGL(ia::k_select_count, dim3(g), dim3(ia::kWG), 0, s, votes, sh.n_boxes, chunk, hist, n_bins,
                     top_k, cnt, ev);
  hipLaunchKernelGGL(ia::k_select_write, dim3(g), dim3(ia::kWG), 0, s, votes, sh.n_boxes, chunk, hist, n_bins,
                     top_k, cnt, tmp_idx, &persistent(c)->done_counter, parents, sh, out_boxes, out_index,
                     out_votes, ev, v_min_stop);
  IA_HIP(c, hipGetLastError());
  return IA_OK;
}

// boxes per workgroup of the vote kernel for a level of n_boxes boxes per
// event over n_ev events: large levels and large batches use one lane per
// box; small levels of few events split each chunk's hits over 2 or 4 waves
// so that the device gets enough workgroups
int32_t vote_tile(const ia_ctx* c, uint32_t n_boxes, int32_t n_ev) {
  if (c->tile_override) return c->tile_override;
  for (const auto& t : c->tuned)
    if (t.first == n_boxes) return t.second;
  if (n_boxes >= (1u << 19) || uint64_t(n_boxes) * uint64_t(std::max(n_ev, 1)) >= (uint64_t(1) << 22)) return 256;
  return 128;
}

// the exclusion and inclusion proofs of the (triple, hit) classification:
// on unless switched off (then every stereo pair is evaluated per box)
int32_t use_filter(const ia_ctx* c) { return c->filter_mode >= 0 ? c->filter_mode : 1; }

ia::EvView single_view(int32_t n_hits) {
  ia::EvView v{};
  v.off = nullptr;
  v.n_single = n_hits;
  return v;
}

// launches the (triple, hit) classification of a level for n_ev events
// (tlb and tn2 must be zero on entry; the kernel adds to them).  The hits
// are split over enough groups (grid z) to give the device about 2048
// workgroups when the triples alone do not.
ia_status launch_classify(ia_ctx* c, const HitRec* recs, const ia::EvView& vw, int32_t n_ev, int32_t max_hits,
                          const BoxD* par, const Shape& sh, uint8_t* flags, int32_t* tlb, int32_t* tn2,
                          const EventState* ev, hipStream_t s, bool f32, float slack32,
                          const uint8_t* pflags = nullptr, const ia::ParentE* pe = nullptr, bool exact = false) {
  const uint32_t n_tr = sh.n_parents * sh.m012;
  const uint32_t gx = (n_tr + 63) / 64;
  const int64_t base = int64_t(gx) * std::max(1, n_ev);
  const int32_t max_groups = std::max(1, (max_hits + ia::kWG / 64 - 1) / (ia::kWG / 64));
  const int32_t hg = static_cast<int32_t>(std::min<int64_t>(std::max<int64_t>(1, 2048 / base), std::min(max_groups, 64)));
  const dim3 g(gx, n_ev, hg);
  // the class proofs enclose the FP64 ApproxPhi form of d^Ax: with the
  // exact Phi, and at FP32 levels (the whole predicate in FP32), every
  // stereo pair is evaluated box by box
  const int32_t filt = (exact || f32) ? 0 : use_filter(c);
  unsigned long long* wk = persistent(c)->work;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profiling) {
    IA_HIP(c, hipEventCreate(&e0));
    IA_HIP(c, hipEventCreate(&e1));
    IA_HIP(c, hipEventRecord(e0, s));
  }
  const dim3 b(ia::kWG);
  if (c->count_work) {
    if (f32)
      hipLaunchKernelGGL((ia::k_classify<true, true>), g, b, 0, s, recs, vw, par, sh, flags, tlb, tn2, filt, ev,
                         slack32, pflags, pe, wk);
    else
      hipLaunchKernelGGL((ia::k_classify<false, true>), g, b, 0, s, recs, vw, par, sh, flags, tlb, tn2, filt, ev,
                         slack32, pflags, pe, wk);
  } else if (f32) {
    hipLaunchKernelGGL((ia::k_classify<true, false>), g, b, 0, s, recs, vw, par, sh, flags, tlb, tn2, filt, ev,
                       slack32, pflags, pe, nullptr);
  } else {
    hipLaunchKernelGGL((ia::k_classify<false, false>), g, b, 0, s, recs, vw, par, sh, flags, tlb, tn2, filt, ev,
                       slack32, pflags, pe, nullptr);
  }
  if (c->profiling) {
    IA_HIP(c, hipEventRecord(e1, s));
    c->marks.push_back({e0, e1, f32, sh.n_boxes, IA_KERNEL_CLASSIFY});
  }
  IA_HIP(c, hipGetLastError());
  // the pairs left to the enclosure passes, compacted per chunk of flags:
  // the largest chunk that still gives about 2048 workgroups
  const int64_t n_pairs = int64_t(n_tr) * std::max(0, max_hits);
  // pair indices and the per-event record counts and offsets are 32-bit
  if (n_pairs >= (int64_t(1) << 31)) return fail(c, IA_ERR_OVERFLOW, "level has 2^31 or more (triple, hit) pairs");
  if (filt && n_pairs > 0) {
    int32_t per = ia::kDeferPer;
    while (per > 1 && (n_pairs * std::max(1, n_ev)) / (int64_t(per) * ia::kWG) < 2048) per /= 2;
    const dim3 gd(static_cast<uint32_t>((n_pairs + int64_t(per) * ia::kWG - 1) / (int64_t(per) * ia::kWG)), n_ev);
    hipEvent_t d0 = nullptr, d1 = nullptr;
    if (c->profiling) {
      IA_HIP(c, hipEventCreate(&d0));
      IA_HIP(c, hipEventCreate(&d1));
      IA_HIP(c, hipEventRecord(d0, s));
    }
    if (c->count_work) {
      if (f32)
        hipLaunchKernelGGL((ia::k_classify_defer<true, true>), gd, b, 0, s, recs, vw, par, sh, flags, tlb, tn2, per,
                           ev, slack32, wk);
      else
        hipLaunchKernelGGL((ia::k_classify_defer<false, true>), gd, b, 0, s, recs, vw, par, sh, flags, tlb, tn2, per,
                           ev, slack32, wk);
    } else if (f32) {
      hipLaunchKernelGGL((ia::k_classify_defer<true, false>), gd, b, 0, s, recs, vw, par, sh, flags, tlb, tn2, per,
                         ev, slack32, nullptr);
    } else {
      hipLaunchKernelGGL((ia::k_classify_defer<false, false>), gd, b, 0, s, recs, vw, par, sh, flags, tlb, tn2, per,
                         ev, slack32, nullptr);
    }
    if (c->profiling) {
      IA_HIP(c, hipEventRecord(d1, s));
      c->marks.push_back({d0, d1, f32, sh.n_boxes, IA_KERNEL_CLASSIFY_DEFER});
    }
    IA_HIP(c, hipGetLastError());
  }
  return IA_OK;
}

// launches the vote kernel for n_ev events, bracketed by events when profiling
struct VoteIn {                   // per-level inputs of the vote kernel
  const uint8_t* flags;
  const int32_t* tlb;
  const int32_t* tn2;
  const int32_t* live_list;       // null: every tile of the level
  int32_t only_unstaged;          // vote only events whose records did not fit
};

template <bool F32, bool EX>
void launch_vote_tile(int32_t bx, dim3 g, hipStream_t s, const HitRec* recs, const ia::EvView& vw, const BoxD* par,
                      const Shape& sh, uint16_t* votes, uint32_t* hist, uint32_t* st, const EventState* ev,
                      const VoteIn& in, int32_t* wg_max, unsigned long long* wk, float slack32) {
  switch (bx) {
    case 256:
      hipLaunchKernelGGL((ia::k_vote<256, F32, EX>), g, dim3(ia::kWG), 0, s, recs, vw, par, sh, votes, hist, st, ev,
                         in.flags, in.tlb, in.tn2, in.live_list, wg_max, wk, slack32, in.only_unstaged);
      break;
    case 128:
      hipLaunchKernelGGL((ia::k_vote<128, F32, EX>), g, dim3(ia::kWG), 0, s, recs, vw, par, sh, votes, hist, st, ev,
                         in.flags, in.tlb, in.tn2, in.live_list, wg_max, wk, slack32, in.only_unstaged);
      break;
    default:
      hipLaunchKernelGGL((ia::k_vote<64, F32, EX>), g, dim3(ia::kWG), 0, s, recs, vw, par, sh, votes, hist, st, ev,
                         in.flags, in.tlb, in.tn2, in.live_list, wg_max, wk, slack32, in.only_unstaged);
      break;
  }
}

ia_status launch_vote(ia_ctx* c, const HitRec* recs, const ia::EvView& vw, int32_t n_ev, const BoxD* par,
                      const Shape& sh, uint16_t* votes, uint32_t* hist, const EventState* ev, const VoteIn& in,
                      int32_t* wg_max, hipStream_t s, bool f32, float slack32, int32_t* tile_used = nullptr,
                      bool exact = false) {
  const int32_t bx = vote_tile(c, sh.n_boxes, n_ev);
  // workgroups stride over the tiles: with a live list, about kVoteGroups in
  // all (most tiles of a pruned level are not live); otherwise one per tile
  // up to a cap
  const uint32_t n_tiles = (sh.n_boxes + bx - 1) / bx;
  uint32_t grid = std::min<uint32_t>(n_tiles, 16384u);
  if (in.live_list)
    grid = std::max<uint32_t>(1, std::min<uint32_t>(n_tiles, (kVoteGroups + n_ev - 1) / std::max(1, n_ev)));
  if (tile_used) *tile_used = bx;
  // the fallback for events whose records did not fit (in.only_unstaged)
  // extends the level's vote mark instead of adding a launch of its own, so
  // that a level's vote counts once
  const bool extend = in.only_unstaged && c->profiling && !c->marks.empty() &&
                      c->marks.back().kind == IA_KERNEL_VOTE;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profiling) {
    if (!extend) IA_HIP(c, hipEventCreate(&e0));
    IA_HIP(c, hipEventCreate(&e1));
    if (!extend) IA_HIP(c, hipEventRecord(e0, s));
  }
  uint32_t* st = &persistent(c)->status;
  unsigned long long* wk = persistent(c)->work;
  const dim3 g(grid, n_ev);
  if (f32) launch_vote_tile<true, false>(bx, g, s, recs, vw, par, sh, votes, hist, st, ev, in, wg_max, wk, slack32);
  else if (exact) launch_vote_tile<false, true>(bx, g, s, recs, vw, par, sh, votes, hist, st, ev, in, wg_max, wk, slack32);
  else launch_vote_tile<false, false>(bx, g, s, recs, vw, par, sh, votes, hist, st, ev, in, wg_max, wk, slack32);
  if (c->profiling) {
    IA_HIP(c, hipEventRecord(e1, s));
    if (extend) {
      (void)hipEventDestroy(c->marks.back().e1);
      c->marks.back().e1 = e1;
    } else {
      c->marks.push_back({e0, e1, f32, sh.n_boxes, IA_KERNEL_VOTE});
    }
  }
  IA_HIP(c, hipGetLastError());
  return IA_OK;
}

struct RecIn {                    // per-level staged-record buffers
  int32_t* live_tri;
  int32_t* rec_off;
  int32_t* rec_fill;
  void* rec;
  ia::TriFrame* tfr;
  int32_t* live_off;              // n_ev + 1 offsets of the events' live tiles in one list
  int64_t* stage_off;             // n_ev + 1 offsets of the events' (live triple, hit) pairs
};

// stages the class-2 records of a level; first lays out the batch's stage
// items and live vote tiles in one list each (k_live_offsets), which the
// vote kernel then uses too
void launch_stage(const HitRec* recs, const ia::EvView& vw, int32_t n_ev, const BoxD* par, const Shape& sh,
                  const uint8_t* flags, const RecIn& r, const EventState* ev, hipStream_t s, bool f32,
                  float slack32) {
  hipLaunchKernelGGL(ia::k_live_offsets, dim3(1), dim3(ia::kWG), 0, s, ev, vw, n_ev, r.live_off, r.stage_off);
  // no more workgroups than the level's items could fill: at most n_ev x
  // triples x max_hits (live triple, hit) items, kStageBatch x kWG each, so
  // that small batches do not start thousands of empty workgroups
  int64_t groups = kVoteGroups;
  if (vw.max_hits > 0) {
    const int64_t items = int64_t(std::max(1, n_ev)) * sh.n_parents * sh.m012 * vw.max_hits;
    const int64_t per = int64_t(ia::kStageBatch) * ia::kWG;
    groups = std::max<int64_t>(1, std::min<int64_t>(kVoteGroups, (items + per - 1) / per));
  }
  const dim3 g(static_cast<uint32_t>(groups), 1);
  if (f32)
    hipLaunchKernelGGL((ia::k_stage<true>), g, dim3(ia::kWG), 0, s, recs, vw, par, sh, flags, r.live_tri, r.rec_off,
                       r.rec_fill, r.rec, r.tfr, r.stage_off, n_ev, slack32);
  else
    hipLaunchKernelGGL((ia::k_stage<false>), g, dim3(ia::kWG), 0, s, recs, vw, par, sh, flags, r.live_tri, r.rec_off,
                       r.rec_fill, r.rec, r.tfr, r.stage_off, n_ev, slack32);
}

template <bool F32, bool EX>
void launch_vote_rec_tile(int32_t bx, dim3 g, hipStream_t s, const ia::EvView& vw, int32_t n_ev, const BoxD* par,
                          const Shape& sh, uint16_t* votes, uint32_t* hist, uint32_t* st, const EventState* ev,
                          const VoteIn& in, const RecIn& r, int32_t* wg_max, unsigned long long* wk) {
  switch (bx) {
    case 256:
      hipLaunchKernelGGL((ia::k_vote_rec<256, F32, EX>), g, dim3(ia::kWG), 0, s, vw, par, sh, votes, hist, st, ev, in.tlb,
                         in.tn2, in.live_list, r.live_off, n_ev, r.rec_off, r.rec, r.tfr, wg_max, wk);
      break;
    case 128:
      hipLaunchKernelGGL((ia::k_vote_rec<128, F32, EX>), g, dim3(ia::kWG), 0, s, vw, par, sh, votes, hist, st, ev, in.tlb,
                         in.tn2, in.live_list, r.live_off, n_ev, r.rec_off, r.rec, r.tfr, wg_max, wk);
      break;
    default:
      hipLaunchKernelGGL((ia::k_vote_rec<64, F32, EX>), g, dim3(ia::kWG), 0, s, vw, par, sh, votes, hist, st, ev, in.tlb,
                         in.tn2, in.live_list, r.live_off, n_ev, r.rec_off, r.rec, r.tfr, wg_max, wk);
      break;
  }
}

// the IV levels' vote (k_vote_iv) over the listed live tiles of n_ev events
// (live_list null: every tile), bracketed by events when profiling
ia_status launch_vote_iv(ia_ctx* c, const HitRec* recs, const ia::EvView& vw, int32_t n_ev, const BoxD* par,
                         const Shape& sh, const uint8_t* flags, uint16_t* votes, uint32_t* hist,
                         const EventState* ev, const int32_t* tlb, const int32_t* tn2, const int32_t* live_list,
                         const int32_t* live_off, int32_t* wg_max, hipStream_t s) {
  const uint32_t n_tiles = (sh.n_boxes + ia::kWG - 1) / ia::kWG;
  const uint32_t grid = static_cast<uint32_t>(
      std::max<int64_t>(1, std::min<int64_t>(int64_t(n_tiles) * std::max(1, n_ev), kVoteGroups)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profiling) {
    IA_HIP(c, hipEventCreate(&e0));
    IA_HIP(c, hipEventCreate(&e1));
    IA_HIP(c, hipEventRecord(e0, s));
  }
  hipLaunchKernelGGL(ia::k_vote_iv, dim3(grid), dim3(ia::kWG), 0, s, recs, vw, par, sh, flags, votes, hist,
                     &persistent(c)->status, ev, tlb, tn2, live_list, live_off, n_ev, wg_max, persistent(c)->work);
  if (c->profiling) {
    IA_HIP(c, hipEventRecord(e1, s));
    c->marks.push_back({e0, e1, false, sh.n_boxes, IA_KERNEL_VOTE});
  }
  IA_HIP(c, hipGetLastError());
  return IA_OK;
}

// the record-based vote for n_ev events (bracketed by events when profiling)
ia_status launch_vote_rec(ia_ctx* c, const ia::EvView& vw, int32_t n_ev, const BoxD* par, const Shape& sh,
                          uint16_t* votes, uint32_t* hist, const EventState* ev, const VoteIn& in, const RecIn& r,
                          int32_t* wg_max, hipStream_t s, bool f32, bool exact = false) {
  const int32_t bx = vote_tile(c, sh.n_boxes, n_ev);
  const uint32_t n_tiles = (sh.n_boxes + bx - 1) / bx;
  // the batch's live tiles in one list (laid out by launch_stage), shared by
  // all workgroups
  const uint32_t grid = static_cast<uint32_t>(
      std::max<int64_t>(1, std::min<int64_t>(int64_t(n_tiles) * std::max(1, n_ev), kVoteGroups)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profiling) {
    IA_HIP(c, hipEventCreate(&e0));
    IA_HIP(c, hipEventCreate(&e1));
    IA_HIP(c, hipEventRecord(e0, s));
  }
  uint32_t* st = &persistent(c)->status;
  unsigned long long* wk = persistent(c)->work;
  const dim3 g(grid, 1);
  if (f32) launch_vote_rec_tile<true, false>(bx, g, s, vw, n_ev, par, sh, votes, hist, st, ev, in, r, wg_max, wk);
  else if (exact) launch_vote_rec_tile<false, true>(bx, g, s, vw, n_ev, par, sh, votes, hist, st, ev, in, r, wg_max, wk);
  else launch_vote_rec_tile<false, false>(bx, g, s, vw, n_ev, par, sh, votes, hist, st, ev, in, r, wg_max, wk);
  if (c->profiling) {
    IA_HIP(c, hipEventRecord(e1, s));
    c->marks.push_back({e0, e1, f32, sh.n_boxes, IA_KERNEL_VOTE});
  }
  IA_HIP(c, hipGetLastError());
  return IA_OK;
}

// scratch layout of one chunk of ia_find_helices (byte offsets into the
// arena): per-event slices of every array, sized for events of max_hits hits
struct FindLayout {
  size_t win, off, recs, votes, hist, lbh, selA, selB, range, sel_idx, sel_v, ev, part, flags, tlb, tn2, wg_max, live,
      live_tri, rec_off, rec_fill, tfr, rec, pflags, pe, live_off, stage_off, emask, total;
  int64_t flag_stride, tri_stride, votes_stride, rec_stride, pflag_stride;
  int32_t hist_stride, wg_stride, part_stride, n_part, emask_stride;
};

// rec_per_event: staged records per event (0: every (triple, hit) pair)
void layout_find(int64_t max_level_boxes, int64_t max_triples, int32_t top_k, int32_t max_hits, int32_t n_ev,
                 int64_t n_hits_total, FindLayout* L, int64_t rec_per_event = 0) {
  L->n_part = est_parts(static_cast<uint32_t>(max_level_boxes));
  L->votes_stride = max_level_boxes;
  L->hist_stride = max_hits + 2;
  L->flag_stride = max_triples * int64_t(std::max(0, max_hits));
  L->tri_stride = max_triples;
  L->pflag_stride = int64_t(std::max(1, top_k)) * int64_t(std::max(0, max_hits));
  L->rec_stride = rec_per_event > 0 ? rec_per_event : std::max<int64_t>(1, max_triples * int64_t(std::max(0, max_hits)));
  L->wg_stride = static_cast<int32_t>((max_level_boxes + 63) / 64);
  L->part_stride = ia::kEstQ * L->n_part;
  L->emask_stride = (L->n_part + 31) / 32;
  const size_t E = size_t(std::max(1, n_ev));
  size_t off = align_up(sizeof(Persistent));
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes + 1);
    return o;
  };
  L->win = take(sizeof(BoxD) * E);
  L->off = take(sizeof(int32_t) * (E + 1));
  L->recs = take(sizeof(HitRec) * size_t(std::max<int64_t>(1, n_hits_total)));
  L->votes = take(sizeof(uint16_t) * size_t(L->votes_stride) * E);
  L->hist = take(sizeof(uint32_t) * size_t(L->hist_stride) * E);
  L->lbh = take(sizeof(uint32_t) * size_t(L->hist_stride) * E);
  L->selA = take(sizeof(BoxD) * size_t(top_k) * E);
  L->selB = take(sizeof(BoxD) * size_t(top_k) * E);
  L->range = take(sizeof(BoxD));
  L->sel_idx = take(sizeof(int64_t) * size_t(top_k) * E);
  L->sel_v = take(sizeof(uint16_t) * size_t(top_k) * E);
  L->ev = take(sizeof(EventState) * E);
  L->part = take(sizeof(double) * size_t(L->part_stride) * E);
  L->emask = take(sizeof(uint32_t) * size_t(L->emask_stride) * E);
  L->flags = take(size_t(L->flag_stride) * E);
  L->tlb = take(sizeof(int32_t) * size_t(L->tri_stride) * E);
  L->tn2 = take(sizeof(int32_t) * size_t(L->tri_stride) * E);
  L->wg_max = take(sizeof(int32_t) * size_t(L->wg_stride) * E);
  L->live = take(sizeof(int32_t) * size_t(L->wg_stride) * E);
  L->live_tri = take(sizeof(int32_t) * size_t(L->tri_stride) * E);
  L->rec_off = take(sizeof(int32_t) * size_t(L->tri_stride) * E);
  L->rec_fill = take(sizeof(int32_t) * size_t(L->tri_stride) * E);
  L->tfr = take(sizeof(ia::TriFrame) * size_t(L->tri_stride) * E);
  L->rec = take(sizeof(ia::RecD) * size_t(L->rec_stride) * E);
  L->pflags = take(size_t(L->pflag_stride) * E);
  L->pe = take(sizeof(ia::ParentE) * size_t(L->pflag_stride) * E);
  L->live_off = take(sizeof(int32_t) * (E + 1));
  L->stage_off = take(sizeof(int64_t) * (E + 1));
  L->total = off;
}

struct SchedShapes {
  Shape sh0, shr;
  int64_t max_boxes, max_triples;
};

// selection size of a schedule: the window schedule keeps the first
// max-vote box only (its levels need the maximum and the max-vote set)
int32_t sched_k(const ia_schedule* sc) { return sc->mode == IA_SCHED_WINDOW ? 1 : sc->top_k; }

bool sched_shapes(const ia_schedule* sc, SchedShapes* S) {
  if (!make_shape(sc->bins, 1, &S->sh0)) return false;
  S->max_boxes = S->sh0.n_boxes;
  S->max_triples = S->sh0.m012;
  if (sc->mode == IA_SCHED_WINDOW) {
    if (sc->n_refine < 0 || sc->n_refine >= IA_MAX_LEVELS) return false;
    S->shr = S->sh0;
    for (int l = 1; l <= sc->n_refine; ++l) {
      Shape sh;
      if (!make_shape(sc->lbins[l], 1, &sh)) return false;
      S->max_boxes = std::max<int64_t>(S->max_boxes, sh.n_boxes);
      S->max_triples = std::max<int64_t>(S->max_triples, sh.m012);
    }
    return true;
  }
  if (!make_shape(sc->split, std::max(1, sc->top_k), &S->shr)) return false;
  S->max_boxes = std::max<int64_t>(S->sh0.n_boxes, S->shr.n_boxes);
  S->max_triples = std::max<int64_t>(int64_t(S->sh0.n_parents) * S->sh0.m012, int64_t(S->shr.n_parents) * S->shr.m012);
  return true;
}

ia_status check_sched(ia_ctx* c, const ia_schedule* sc) {
  if (sc->n_refine < 0 || sc->n_refine >= IA_MAX_LEVELS) return fail(c, IA_ERR_INVALID, "n_refine %d", sc->n_refine);
  if (!(sc->disk >= 0.0) || !std::isfinite(sc->disk)) return fail(c, IA_ERR_INVALID, "disk %g", sc->disk);
  if (sc->mode != IA_SCHED_TOPK && sc->mode != IA_SCHED_WINDOW) return fail(c, IA_ERR_INVALID, "mode %d", sc->mode);
  if (sc->forward != 0 && sc->forward != 1) return fail(c, IA_ERR_INVALID, "forward %d", sc->forward);
  if (sc->mode == IA_SCHED_WINDOW) {
    if (sc->move_level < -1 || sc->move_level >= sc->n_refine)
      return fail(c, IA_ERR_INVALID, "move_level %d outside [-1, n_refine)", sc->move_level);
    if (sc->wdrop < 0 || sc->wdrop > 65535) return fail(c, IA_ERR_INVALID, "wdrop %d", sc->wdrop);
    if (sc->hitsel != 0 && sc->hitsel != 1) return fail(c, IA_ERR_INVALID, "hitsel %d", sc->hitsel);
    for (int l = 1; l <= sc->n_refine; ++l)
      for (int j = 0; j < 5; ++j)
        if (sc->lbins[l][j] < 1) return fail(c, IA_ERR_INVALID, "lbins[%d][%d] = %d < 1", l, j, sc->lbins[l][j]);
    for (int j = 0; j < 5; ++j)
      if (!std::isfinite(sc->range.lo[j]) || !std::isfinite(sc->range.hi[j]))
        return fail(c, IA_ERR_INVALID, "range dimension %d is not finite", j);
  } else if (sc->top_k < 1 || sc->top_k > kMaxTopK) {
    return fail(c, IA_ERR_INVALID, "top_k %d", sc->top_k);
  }
  if (sc->n_helix_max < 0) return fail(c, IA_ERR_INVALID, "n_helix_max %d", sc->n_helix_max);
  if (!(sc->hitfind_scale >= 0.0)) return fail(c, IA_ERR_INVALID, "hitfind_scale");
  for (int j = 0; j < 5; ++j)
    if (!(sc->range.lo[j] <= sc->range.hi[j])) return fail(c, IA_ERR_INVALID, "range dimension %d: lo > hi", j);
  for (int l = 0; l <= sc->n_refine; ++l)
    if (sc->prec[l] != IA_FP64 && sc->prec[l] != IA_FP32 && sc->prec[l] != IA_FP64X && sc->prec[l] != IA_IV)
      return fail(c, IA_ERR_INVALID, "precision %d at level %d", sc->prec[l], l);
  if (!(sc->fp32_slack >= 0.0 && sc->fp32_slack <= 1e-3))
    return fail(c, IA_ERR_INVALID, "fp32_slack %g outside [0, 1e-3]", sc->fp32_slack);
  return IA_OK;
}

// The window schedule (ia_schedule, IA_SCHED_WINDOW) for a chunk of E
// events whose hits are prepared: per pass, every level votes one grid over
// the event's window (the range at level 0), keeps only the first max-vote
// box (so that its pruning threshold is the largest lower bound), reduces the
// estimate and the union of all max-vote boxes, and builds the next window
// (after move_level: the closest hit, the hull of the moved corners, and the
// hits re-prepared about the new reference point).  The last level runs hit
// finding and writes the helix.
ia_status run_window(ia_ctx* c, const double* hits, ia::EvView vw, int32_t E, int32_t cmax, const SchedShapes& S,
                     const ia_schedule* sc, float slack32, bool may_overflow, const FindLayout& L, HitRec* recs,
                     uint16_t* votes, uint32_t* hist, BoxD* sel, BoxD* range, int64_t* sel_idx, uint16_t* sel_v,
                     EventState* ev, double* part, uint8_t* flags, uint8_t* pflags, ia::ParentE* pe, int32_t* tlb,
                     int32_t* tn2, uint32_t* lbh, int32_t* wg_max, int32_t* live, const RecIn& rin,
                     int32_t* assigned, ia::HelixOut* out, int32_t* n_out, int32_t pass0, int32_t pass1,
                     hipStream_t s) {
  BoxD* win = reinterpret_cast<BoxD*>(c->arena + L.win);
  // chunk masks of the sparse estimate: zero on entry, and k_est_final
  // clears what it read
  uint32_t* emask = reinterpret_cast<uint32_t*>(c->arena + L.emask);
  {
    const uint32_t n_words = static_cast<uint32_t>(L.emask_stride) * static_cast<uint32_t>(E);
    hipLaunchKernelGGL(ia::k_fill_u32, dim3(std::min<uint32_t>((n_words + 255) / 256, 65535)), dim3(256), 0, s, emask,
                       n_words, 0u);
  }
  BoxD rb;
  std::memcpy(&rb, &sc->range, sizeof rb);
  const int32_t pg = std::max(1, (cmax + 255) / 256);
  const int32_t max_per_event = vw.max_out;
  (void)max_per_event;
  for (int32_t pass = pass0; pass < pass1; ++pass) {
    // every pass starts about the origin
    if (pass > 0 && (sc->move_level >= 0 || sc->hitsel))
      hipLaunchKernelGGL(ia::k_reframe, dim3(pg, E), dim3(ia::kWG), 0, s, hits, vw, recs, ev, 1);
    const BoxD* par = range;
    Shape sh = S.sh0;
    vw.par_stride = 0;
    for (int32_t lev = 0; lev <= sc->n_refine; ++lev) {
      const bool f32 = sc->prec[lev] == IA_FP32, exact = sc->prec[lev] == IA_FP64X, iv = sc->prec[lev] == IA_IV;
      vw.fwd = sc->forward;     // per event: hits ahead about the origin, origin behind after a move
      const bool use_pf = lev > 0 && use_filter(c) && c->parent_filter && !exact && !f32 && !iv;
      if (use_pf) {
        const int64_t n_pairs = int64_t(sh.n_parents) * std::max(1, cmax);
        const dim3 gp(static_cast<uint32_t>(std::min<int64_t>((n_pairs + ia::kWG - 1) / ia::kWG, 65535)), E);
        if (f32)
          hipLaunchKernelGGL((ia::k_parent_filter<true>), gp, dim3(ia::kWG), 0, s, recs, vw, par, sh, pflags, ev,
                             slack32, nullptr);
        else
          hipLaunchKernelGGL((ia::k_parent_filter<false>), gp, dim3(ia::kWG), 0, s, recs, vw, par, sh, pflags, ev,
                             slack32, pe);
      }
      {
        const ia_status cs = launch_classify(c, recs, vw, E, cmax, par, sh, flags, tlb, tn2, ev, s, f32, slack32,
                                             use_pf ? pflags : nullptr, (use_pf && !f32) ? pe : nullptr, exact || iv);
        if (cs != IA_OK) return cs;
      }
      const int32_t vt = iv ? ia::kWG : vote_tile(c, sh.n_boxes, E);
      // probe: vote the triples with the largest upper bounds first; the
      // largest vote found raises the level's pruning threshold
      const bool probe = c->prune == 2 && !iv;
      if (probe) {
        hipLaunchKernelGGL(ia::k_threshold, dim3(1, E), dim3(ia::kWG), 0, s, tlb, tn2, lbh, vw, sh, 1, 1, 0, vt, ev,
                           live, wg_max, rin.live_tri, rin.rec_off, rin.rec_fill, L.rec_stride, 0, 1);
        launch_stage(recs, vw, E, par, sh, flags, rin, ev, s, f32, slack32);
        const VoteIn pin{flags, tlb, tn2, live, 1};
        const ia_status st = launch_vote_rec(c, vw, E, par, sh, votes, nullptr, ev, pin, rin, wg_max, s, f32, exact);
        if (st != IA_OK) return st;
      }
      hipLaunchKernelGGL(ia::k_threshold, dim3(1, E), dim3(ia::kWG), 0, s, tlb, tn2, lbh, vw, sh, 1, c->prune, 0,
                         vt, ev, live, wg_max, rin.live_tri, rin.rec_off, rin.rec_fill,
                         iv ? INT64_MAX : L.rec_stride, lev < sc->n_refine ? sc->wdrop : 0, probe ? 2 : 0);
      int32_t bx = vt;
      if (iv) {
        hipLaunchKernelGGL(ia::k_live_offsets, dim3(1), dim3(ia::kWG), 0, s, ev, vw, E, rin.live_off, rin.stage_off);
        const ia_status st = launch_vote_iv(c, recs, vw, E, par, sh, flags, votes, hist, ev, tlb, tn2, live,
                                            rin.live_off, wg_max, s);
        if (st != IA_OK) return st;
      } else {
        launch_stage(recs, vw, E, par, sh, flags, rin, ev, s, f32, slack32);
        const VoteIn in{flags, tlb, tn2, live, 1};
        ia_status st = launch_vote_rec(c, vw, E, par, sh, votes, hist, ev, in, rin, wg_max, s, f32, exact);
        if (st != IA_OK) return st;
        if (may_overflow) {
          st = launch_vote(c, recs, vw, E, par, sh, votes, hist, ev, in, wg_max, s, f32, slack32, &bx, exact);
          if (st != IA_OK) return st;
        }
      }
      const uint32_t n_wg = (sh.n_boxes + bx - 1) / bx;
      hipLaunchKernelGGL(ia::k_select_wg, dim3(1, E), dim3(ia::kWG), 0, s, votes, vw, hist, wg_max, n_wg, bx, par,
                         sh, sel, sel_idx, sel_v, ev, lev == 0 ? std::max(sc->v_min, 0) : 0, tlb, tn2, 1);
      const int32_t n_part = est_parts(sh.n_boxes);
      const uint32_t eper = est_per(n_part, E);
      const dim3 gpart((n_part + eper - 1) / eper, E);
      // one track at a time: the phi0 run of the first max-vote box
      hipLaunchKernelGGL(ia::k_phi_occ, gpart, dim3(ia::kWG), 0, s, votes, sh, sel_v, ev, vw, wg_max, bx,
                         static_cast<uint32_t>(n_part), eper);
      hipLaunchKernelGGL(ia::k_phi_run, dim3(1, E), dim3(64), 0, s, par, sh, sel_idx, ev, vw);
      // the max-vote boxes' sums, over the chunks of the live tiles only
      // (sparse: the other chunks are the identity, marked by clear bits)
      hipLaunchKernelGGL(ia::k_est_partial, dim3(std::min(kEstGroups, n_part), E), dim3(ia::kWG), 0, s, par, sh,
                         votes, sel, sel_v, part, vw, ev, wg_max, bx, static_cast<uint32_t>(n_part), eper, 1, live,
                         emask, L.emask_stride);
      if (lev == sc->n_refine) {
        // bit 0: the forward test, applied while the event's frame is the
        // origin's; bit 1: the exact Phi of the last level
        const int32_t fwd_hf = (sc->forward ? 1 : 0) | (exact ? 2 : 0);
        hipLaunchKernelGGL(ia::k_est_final, dim3(1, E), dim3(ia::kWG), 0, s, part, n_part, sel, sel_v,
                           static_cast<ia::EstimateOut*>(nullptr), ev, recs, vw, sc->hitfind_scale, assigned, out,
                           n_out, fwd_hf, emask, L.emask_stride);
        IA_HIP(c, hipGetLastError());
        break;
      }
      hipLaunchKernelGGL(ia::k_est_final, dim3(1, E), dim3(ia::kWG), 0, s, part, n_part, sel, sel_v,
                         static_cast<ia::EstimateOut*>(nullptr), ev, static_cast<HitRec*>(nullptr), vw, 0.0,
                         static_cast<int32_t*>(nullptr), static_cast<ia::HelixOut*>(nullptr),
                         static_cast<int32_t*>(nullptr), 0, emask, L.emask_stride);
      if (sc->hitsel)
        hipLaunchKernelGGL(ia::k_hit_select, dim3(pg, E), dim3(ia::kWG), 0, s, recs, vw, ev, sc->hitfind_scale,
                           (vw.fwd ? 1 : 0) | (exact ? 2 : 0));
      const bool mv = lev == sc->move_level;
      if (mv) hipLaunchKernelGGL(ia::k_closest, dim3(1, E), dim3(ia::kWG), 0, s, recs, vw, ev);
      // the window's extent over the live tiles: 8 to 32 workgroups per
      // event (at most the part records the arena holds), one record each
      const int32_t n_win = std::min(std::max(kWinGroupsMin, std::min(kWinGroupsMax, kWinTotal / std::max(1, E))),
                                     L.n_part);
      hipLaunchKernelGGL(ia::k_window_partial, dim3(n_win, E), dim3(ia::kWG), 0, s, par, sh, votes, sel, sel_v, part,
                         vw, ev, wg_max, live, bx, sc->wdrop, mv ? 1 : 0);
      ia::Bins5 nb;
      for (int j = 0; j < 5; ++j) nb.m[j] = sc->lbins[lev + 1][j];
      hipLaunchKernelGGL(ia::k_window, dim3(1, E), dim3(ia::kWG), 0, s, part, n_win, par, sh, win, ev, vw, rb, nb,
                         mv ? 1 : 0);
      if (mv) hipLaunchKernelGGL(ia::k_reframe, dim3(pg, E), dim3(ia::kWG), 0, s, hits, vw, recs, ev, 0);
      IA_HIP(c, hipGetLastError());
      if (!make_shape(sc->lbins[lev + 1], 1, &sh)) return fail(c, IA_ERR_OVERFLOW, "level %d too large", lev + 1);
      par = win;
      vw.par_stride = 1;
    }
  }
  return IA_OK;
}

// One chunk of E events through every pass and level.  The chunk's CSR
// offsets (relative to hits_chunk) come from the host (h_off_chunk, copied
// through the pinned ring) or are already on the device (dev_off, then no
// host synchronisation or copy happens: the launches can be captured).
ia_status run_chunk(ia_ctx* c, const double* hits_chunk, const int32_t* h_off_chunk, const int32_t* dev_off,
                    int32_t E, int32_t cmax, int64_t n_tot, const SchedShapes& S, const ia_schedule* sc,
                    float slack32, int64_t rpe, bool may_overflow, ia::HelixOut* out_chunk, int32_t max_per_event,
                    int32_t* n_out_chunk, int32_t* assigned_chunk, hipStream_t s) {
  const int32_t K = sched_k(sc);
  Persistent* ps = persistent(c);
  BoxD rb;
  std::memcpy(&rb, &sc->range, sizeof rb);
  FindLayout L;
  layout_find(S.max_boxes, S.max_triples, K, cmax, E, n_tot, &L, rpe);
  if (L.total > c->arena_bytes) return fail(c, IA_ERR_NOMEM, "chunk layout exceeds scratch");
  char* a = c->arena;
  int32_t* d_off = dev_off ? const_cast<int32_t*>(dev_off) : reinterpret_cast<int32_t*>(a + L.off);
  HitRec* recs = reinterpret_cast<HitRec*>(a + L.recs);
  uint16_t* votes = reinterpret_cast<uint16_t*>(a + L.votes);
  uint32_t* hist = reinterpret_cast<uint32_t*>(a + L.hist);
  BoxD* selA = reinterpret_cast<BoxD*>(a + L.selA);
  BoxD* selB = reinterpret_cast<BoxD*>(a + L.selB);
  BoxD* range = reinterpret_cast<BoxD*>(a + L.range);
  int64_t* sel_idx = reinterpret_cast<int64_t*>(a + L.sel_idx);
  uint16_t* sel_v = reinterpret_cast<uint16_t*>(a + L.sel_v);
  EventState* ev = reinterpret_cast<EventState*>(a + L.ev);
  double* part = reinterpret_cast<double*>(a + L.part);
  uint8_t* flags = reinterpret_cast<uint8_t*>(a + L.flags);
  uint8_t* pflags = reinterpret_cast<uint8_t*>(a + L.pflags);
  ia::ParentE* pe = reinterpret_cast<ia::ParentE*>(a + L.pe);
  int32_t* tlb = reinterpret_cast<int32_t*>(a + L.tlb);
  int32_t* tn2 = reinterpret_cast<int32_t*>(a + L.tn2);
  uint32_t* lbh = reinterpret_cast<uint32_t*>(a + L.lbh);
  int32_t* wg_max = reinterpret_cast<int32_t*>(a + L.wg_max);
  int32_t* live = reinterpret_cast<int32_t*>(a + L.live);
  const RecIn rin{reinterpret_cast<int32_t*>(a + L.live_tri), reinterpret_cast<int32_t*>(a + L.rec_off),
                  reinterpret_cast<int32_t*>(a + L.rec_fill), a + L.rec,
                  reinterpret_cast<ia::TriFrame*>(a + L.tfr), reinterpret_cast<int32_t*>(a + L.live_off),
                  reinterpret_cast<int64_t*>(a + L.stage_off)};
  if (!dev_off) {
    // chunk-relative hit offsets through a pinned slot whose last copy is done
    const uint32_t slot = c->slot_next++ % kOffSlots;
    if (c->slot_used[slot]) IA_HIP(c, hipEventSynchronize(c->slot_done[slot]));
    int32_t* ho = c->pinned + size_t(slot) * kOffSlotInts;
    for (int32_t e = 0; e <= E; ++e) ho[e] = h_off_chunk[e] - h_off_chunk[0];
    IA_HIP(c, hipMemcpyAsync(d_off, ho, sizeof(int32_t) * (size_t(E) + 1), hipMemcpyHostToDevice, s));
    IA_HIP(c, hipEventRecord(c->slot_done[slot], s));
    c->slot_used[slot] = true;
  }
  ia::EvView vw{};
  vw.off = d_off;
  vw.k = K;
  vw.flag_stride = L.flag_stride;
  vw.tri_stride = L.tri_stride;
  vw.rec_stride = L.rec_stride;
  vw.pflag_stride = L.pflag_stride;
  vw.hist_stride = L.hist_stride;
  vw.wg_stride = L.wg_stride;
  vw.part_stride = L.part_stride;
  vw.max_out = max_per_event;
  vw.max_hits = std::max(1, cmax);
  vw.n_total = n_tot;
  const double* hits = hits_chunk;
  int32_t* assigned = assigned_chunk;
  ia::HelixOut* out = out_chunk;
  int32_t* n_out = n_out_chunk;
  const int32_t pg = std::max(1, (cmax + 2 + 255) / 256);
  hipLaunchKernelGGL(ia::k_prep, dim3(pg, E), dim3(256), 0, s, hits, nullptr, vw, recs, hist, lbh, tlb, tn2,
                     &ps->status, &ps->n_bad, ev, n_out, range, rb, assigned, 0.0, 0.0, nullptr);
  vw.disk = sc->disk;
  if (sc->mode == IA_SCHED_WINDOW)
    return run_window(c, hits, vw, E, cmax, S, sc, slack32, may_overflow, L, recs, votes, hist, selA, range, sel_idx,
                      sel_v, ev, part, flags, pflags, pe, tlb, tn2, lbh, wg_max, live, rin, assigned, out, n_out, 0,
                      std::min(sc->n_helix_max, max_per_event), s);
  vw.fwd = sc->forward;
  for (int32_t pass = 0; pass < std::min(sc->n_helix_max, max_per_event); ++pass) {
    const BoxD* par = range;
    Shape sh = S.sh0;
    BoxD* sel = selA;
    vw.par_stride = 0;
    int32_t last_bx = 1;
    for (int32_t lev = 0; lev <= sc->n_refine; ++lev) {
      const bool f32 = sc->prec[lev] == IA_FP32, exact = sc->prec[lev] == IA_FP64X, iv = sc->prec[lev] == IA_IV;
      // refinement levels: the parent-level test first (a hit it excludes
      // is class 0 for all of that parent's triples)
      const bool use_pf = lev > 0 && use_filter(c) && c->parent_filter && !exact && !f32 && !iv;
      if (use_pf) {
        const int64_t n_pairs = int64_t(sh.n_parents) * std::max(1, cmax);
        const dim3 gp(static_cast<uint32_t>(std::min<int64_t>((n_pairs + ia::kWG - 1) / ia::kWG, 65535)), E);
        if (f32)
          hipLaunchKernelGGL((ia::k_parent_filter<true>), gp, dim3(ia::kWG), 0, s, recs, vw, par, sh, pflags, ev,
                             slack32, nullptr);
        else
          hipLaunchKernelGGL((ia::k_parent_filter<false>), gp, dim3(ia::kWG), 0, s, recs, vw, par, sh, pflags, ev,
                             slack32, pe);
      }
      {
        // at FP64 levels the parent's per-sign ranges of d^Ax also decide
        // many pairs in the first stage
        const ia_status cs = launch_classify(c, recs, vw, E, cmax, par, sh, flags, tlb, tn2, ev, s, f32, slack32,
                                             use_pf ? pflags : nullptr, (use_pf && !f32) ? pe : nullptr, exact || iv);
        if (cs != IA_OK) return cs;
      }
      const int32_t vt = iv ? ia::kWG : vote_tile(c, sh.n_boxes, E);
      // the last level feeds only the estimate, which needs the whole
      // max-vote set and the first max-vote box: there the selection keeps
      // one box, so that T is the largest lower bound (a box whose upper
      // bound is below it cannot reach the maximum), and no tie cut applies
      const bool last = lev == sc->n_refine;
      const int32_t k_lev = last ? 1 : K;
      const int32_t ties = last ? 0 : 1;
      hipLaunchKernelGGL(ia::k_threshold, dim3(1, E), dim3(ia::kWG), 0, s, tlb, tn2, lbh, vw, sh, k_lev, c->prune,
                         ties, vt, ev, live, wg_max, rin.live_tri, rin.rec_off, rin.rec_fill,
                         iv ? INT64_MAX : L.rec_stride, 0, 0);
      int32_t bx = vt;
      if (iv) {
        hipLaunchKernelGGL(ia::k_live_offsets, dim3(1), dim3(ia::kWG), 0, s, ev, vw, E, rin.live_off, rin.stage_off);
        const ia_status st = launch_vote_iv(c, recs, vw, E, par, sh, flags, votes, hist, ev, tlb, tn2, live,
                                            rin.live_off, wg_max, s);
        if (st != IA_OK) return st;
      } else {
        launch_stage(recs, vw, E, par, sh, flags, rin, ev, s, f32, slack32);
        const VoteIn in{flags, tlb, tn2, live, 1};
        ia_status st = launch_vote_rec(c, vw, E, par, sh, votes, hist, ev, in, rin, wg_max, s, f32, exact);
        if (st != IA_OK) return st;
        if (may_overflow) {
          st = launch_vote(c, recs, vw, E, par, sh, votes, hist, ev, in, wg_max, s, f32, slack32, &bx, exact);
          if (st != IA_OK) return st;
        }
      }
      last_bx = bx;
      const uint32_t n_wg = (sh.n_boxes + bx - 1) / bx;
      hipLaunchKernelGGL(ia::k_select_wg, dim3(1, E), dim3(ia::kWG), 0, s, votes, vw, hist, wg_max, n_wg, bx, par,
                         sh, sel, sel_idx, sel_v, ev, lev == 0 ? std::max(sc->v_min, 0) : 0, tlb, tn2, k_lev);
      IA_HIP(c, hipGetLastError());
      if (lev == sc->n_refine) break;
      const int32_t k_eff = static_cast<int32_t>(std::min<int64_t>(K, sh.n_boxes));
      if (!make_shape(sc->split, k_eff, &sh)) return fail(c, IA_ERR_OVERFLOW, "split too large");
      par = sel;
      vw.par_stride = K;
      sel = (sel == selA) ? selB : selA;
    }
    const int32_t n_part = est_parts(sh.n_boxes);
    const uint32_t eper = est_per(n_part, E);
    hipLaunchKernelGGL(ia::k_est_partial, dim3((n_part + eper - 1) / eper, E), dim3(ia::kWG), 0, s, par, sh, votes,
                       sel, sel_v, part, vw, ev, wg_max, last_bx, static_cast<uint32_t>(n_part), eper, 0,
                       static_cast<const int32_t*>(nullptr), static_cast<uint32_t*>(nullptr), 0);
    hipLaunchKernelGGL(ia::k_est_final, dim3(1, E), dim3(ia::kWG), 0, s, part, n_part, sel, sel_v,
                       static_cast<ia::EstimateOut*>(nullptr), ev, recs, vw, sc->hitfind_scale, assigned, out, n_out,
                       (sc->forward ? 1 : 0) | (sc->prec[sc->n_refine] == IA_FP64X ? 2 : 0),
                       static_cast<uint32_t*>(nullptr), 0);
    IA_HIP(c, hipGetLastError());
  }
  return IA_OK;
}

}  // namespace

extern "C" {

ia_status ia_ctx_create(ia_ctx** out, int32_t device, size_t scratch_bytes) {
  if (!out) return IA_ERR_INVALID;
  *out = nullptr;
  if (scratch_bytes < 4096) scratch_bytes = 4096;
  ia_ctx* c = new ia_ctx();
  c->device = device;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) { delete c; return IA_ERR_DEVICE; }
  void* p = nullptr;
  e = hipMalloc(&p, scratch_bytes);
  if (e != hipSuccess) { delete c; return IA_ERR_NOMEM; }
  e = hipMemset(p, 0, scratch_bytes);
  if (e != hipSuccess) { (void)hipFree(p); delete c; return IA_ERR_DEVICE; }
  c->arena = static_cast<char*>(p);
  c->arena_bytes = scratch_bytes;
  void* hp = nullptr;
  e = hipHostMalloc(&hp, sizeof(int32_t) * size_t(kOffSlots) * kOffSlotInts, hipHostMallocDefault);
  if (e != hipSuccess) { (void)hipFree(p); delete c; return IA_ERR_NOMEM; }
  c->pinned = static_cast<int32_t*>(hp);
  for (int i = 0; i < kOffSlots; ++i) {
    e = hipEventCreateWithFlags(&c->slot_done[i], hipEventDisableTiming);
    if (e != hipSuccess) { ia_ctx_destroy(c); return IA_ERR_DEVICE; }
  }
  reset_bump(c);
  *out = c;
  return IA_OK;
}

void ia_ctx_destroy(ia_ctx* c) {
  if (!c) return;
  (void)ia_pool_destroy(c);
  for (auto& m : c->marks) {
    (void)hipEventDestroy(m.e0);
    (void)hipEventDestroy(m.e1);
  }
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->arena) (void)hipFree(c->arena);
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (int i = 0; i < kOffSlots; ++i)
    if (c->slot_done[i]) (void)hipEventDestroy(c->slot_done[i]);
  delete c;
}

const char* ia_last_error(const ia_ctx* c) { return c ? c->err.c_str() : g_noalloc_err; }

ia_status ia_ctx_status(ia_ctx* c, uint32_t* flags, int64_t* n_bad) {
  if (!c) return IA_ERR_INVALID;
  IA_HIP(c, hipSetDevice(c->device));
  IA_HIP(c, hipDeviceSynchronize());
  Persistent p;
  IA_HIP(c, hipMemcpy(&p, c->arena, sizeof p, hipMemcpyDeviceToHost));
  if (flags) *flags = p.status;
  if (n_bad) *n_bad = p.n_bad;
  return IA_OK;
}

ia_status ia_ctx_work(ia_ctx* c, int64_t* stereo_box_evals, int64_t* staged_pairs, int64_t* stereo_box_evals_fp32,
                      int64_t* staged_pairs_fp32) {
  if (!c) return IA_ERR_INVALID;
  IA_HIP(c, hipSetDevice(c->device));
  IA_HIP(c, hipDeviceSynchronize());
  Persistent p;
  IA_HIP(c, hipMemcpy(&p, c->arena, sizeof p, hipMemcpyDeviceToHost));
  unsigned long long w[4] = {0, 0, 0, 0};
  for (uint32_t i = 0; i < ia::kWorkSlots; ++i)
    for (int k = 0; k < 4; ++k) w[k] += p.work[i * ia::kWorkSlotU64 + k];
  if (stereo_box_evals) *stereo_box_evals = static_cast<int64_t>(w[0]);
  if (staged_pairs) *staged_pairs = static_cast<int64_t>(w[1]);
  if (stereo_box_evals_fp32) *stereo_box_evals_fp32 = static_cast<int64_t>(w[2]);
  if (staged_pairs_fp32) *staged_pairs_fp32 = static_cast<int64_t>(w[3]);
  return IA_OK;
}

ia_status ia_ctx_classify_work(ia_ctx* c, int64_t counts[16]) {
  if (!c || !counts) return IA_ERR_INVALID;
  IA_HIP(c, hipSetDevice(c->device));
  IA_HIP(c, hipDeviceSynchronize());
  Persistent p;
  IA_HIP(c, hipMemcpy(&p, c->arena, sizeof p, hipMemcpyDeviceToHost));
  for (uint32_t k = 0; k < 2 * ia::kCwN; ++k) {
    unsigned long long w = 0;
    for (uint32_t i = 0; i < ia::kWorkSlots; ++i) w += p.work[i * ia::kWorkSlotU64 + ia::kWorkClassify + k];
    counts[k] = static_cast<int64_t>(w);
  }
  return IA_OK;
}

ia_status ia_ctx_clear_status(ia_ctx* c) {
  if (!c) return IA_ERR_INVALID;
  IA_HIP(c, hipSetDevice(c->device));
  IA_HIP(c, hipDeviceSynchronize());
  Persistent p{};
  IA_HIP(c, hipMemcpy(c->arena, &p, sizeof p, hipMemcpyHostToDevice));
  return IA_OK;
}

ia_status ia_ctx_set_vote_tile(ia_ctx* c, int32_t bx) {
  if (!c) return IA_ERR_INVALID;
  if (bx != 0 && bx != 64 && bx != 128 && bx != 256)
    return fail(c, IA_ERR_INVALID, "vote tile %d not in {0, 64, 128, 256}", bx);
  c->tile_override = bx;
  return IA_OK;
}

ia_status ia_ctx_set_batch(ia_ctx* c, int32_t max_events) {
  if (!c) return IA_ERR_INVALID;
  if (max_events < 1) return fail(c, IA_ERR_INVALID, "max_events %d < 1", max_events);
  c->max_chunk = std::min(max_events, kOffSlotInts - 1);
  return IA_OK;
}

ia_status ia_ctx_set_prefilter(ia_ctx* c, int32_t mode) {
  if (!c) return IA_ERR_INVALID;
  if (mode < -1 || mode > 1) return fail(c, IA_ERR_INVALID, "prefilter mode %d not in {-1, 0, 1}", mode);
  c->filter_mode = mode;
  return IA_OK;
}

ia_status ia_ctx_set_pruning(ia_ctx* c, int32_t enable) {
  if (!c) return IA_ERR_INVALID;
  if (enable < 0 || enable > 2) return fail(c, IA_ERR_INVALID, "pruning mode %d outside 0..2", enable);
  c->prune = enable;
  return IA_OK;
}

ia_status ia_ctx_set_parent_filter(ia_ctx* c, int32_t enable) {
  if (!c) return IA_ERR_INVALID;
  c->parent_filter = enable != 0 ? 1 : 0;
  return IA_OK;
}

ia_status ia_ctx_set_work_counting(ia_ctx* c, int32_t enable) {
  if (!c) return IA_ERR_INVALID;
  c->count_work = enable != 0 ? 1 : 0;
  return IA_OK;
}

ia_status ia_ctx_set_profiling(ia_ctx* c, int32_t enable) {
  if (!c) return IA_ERR_INVALID;
  c->profiling = enable != 0;
  return IA_OK;
}

ia_status ia_ctx_profile_kernels(ia_ctx* c, int64_t n_launches[6], double total_ms[6]) {
  if (!c || !n_launches || !total_ms) return IA_ERR_INVALID;
  IA_HIP(c, hipSetDevice(c->device));
  for (int i = 0; i < 6; ++i) { n_launches[i] = 0; total_ms[i] = 0.0; }
  ia_status st = IA_OK;
  for (auto& m : c->marks) {
    if (st == IA_OK) {
      hipError_t e = hipEventSynchronize(m.e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.e0, m.e1);
      if (e != hipSuccess) st = fail(c, IA_ERR_DEVICE, "profile events: %s", hipGetErrorString(e));
      const int i = 2 * m.kind + (m.f32 ? 1 : 0);
      total_ms[i] += ms;
      ++n_launches[i];
    }
    (void)hipEventDestroy(m.e0);
    (void)hipEventDestroy(m.e1);
  }
  c->marks.clear();
  return st;
}

ia_status ia_ctx_profile_read(ia_ctx* c, int64_t* n_launches, double* total_ms, int64_t* n_launches_fp32,
                              double* total_ms_fp32) {
  int64_t n[6];
  double ms[6];
  const ia_status st = ia_ctx_profile_kernels(c, n, ms);
  if (n_launches) *n_launches = n[2 * IA_KERNEL_VOTE];
  if (total_ms) *total_ms = ms[2 * IA_KERNEL_VOTE];
  if (n_launches_fp32) *n_launches_fp32 = n[2 * IA_KERNEL_VOTE + 1];
  if (total_ms_fp32) *total_ms_fp32 = ms[2 * IA_KERNEL_VOTE + 1];
  return st;
}

ia_status ia_ctx_set_vote_frame(ia_ctx* c, int32_t forward, double xr, double yr, double disk) {
  if (!c) return IA_ERR_INVALID;
  if (forward < 0 || forward > 2) return fail(c, IA_ERR_INVALID, "forward %d", forward);
  if (!std::isfinite(xr) || !std::isfinite(yr)) return fail(c, IA_ERR_INVALID, "reference point not finite");
  if (!(disk >= 0.0) || !std::isfinite(disk)) return fail(c, IA_ERR_INVALID, "disk %g", disk);
  c->vf_disk = disk;
  c->vf_forward = forward;
  c->vf_xr = xr;
  c->vf_yr = yr;
  return IA_OK;
}

ia_status ia_ctx_set_fp32_slack(ia_ctx* c, double slack) {
  if (!c) return IA_ERR_INVALID;
  if (!(slack >= 0.0 && slack <= 1e-3)) return fail(c, IA_ERR_INVALID, "fp32 slack %g outside [0, 1e-3]", slack);
  c->slack32 = ia::ru32(slack);
  return IA_OK;
}

size_t ia_ctx_scratch_needed(const ia_schedule* sc, int32_t max_hits) {
  if (!sc || max_hits < 0) return 0;
  SchedShapes S;
  if (!sched_shapes(sc, &S)) return 0;
  FindLayout L;
  layout_find(S.max_boxes, S.max_triples, std::max(1, sched_k(sc)), max_hits, 1, max_hits, &L);
  return L.total;
}

}  // extern "C"

namespace {

// argument checks shared by ia_vote_level and ia_vote_level_noalloc
ia_status vote_level_args(ia_ctx* c, const ia_hit* d_hits, int32_t n_hits, const ia_box* d_parents,
                          int32_t n_parents, const int32_t split[5], ia_precision prec, const uint16_t* d_votes,
                          Shape* sh) {
  if (n_hits < 0 || n_hits > kMaxHits) return fail(c, IA_ERR_INVALID, "n_hits %d outside [0, %d]", n_hits, kMaxHits);
  if (n_hits > 0 && !d_hits) return fail(c, IA_ERR_INVALID, "d_hits is NULL");
  if (!d_parents || !split || !d_votes) return fail(c, IA_ERR_INVALID, "null pointer argument");
  if (n_parents < 1) return fail(c, IA_ERR_INVALID, "n_parents %d < 1", n_parents);
  if (prec != IA_FP64 && prec != IA_FP32 && prec != IA_FP64X && prec != IA_IV)
    return fail(c, IA_ERR_INVALID, "precision %d unknown", int(prec));
  if (!make_shape(split, n_parents, sh)) return fail(c, IA_ERR_OVERFLOW, "level exceeds 2^31 - 1 boxes");
  return IA_OK;
}

// scratch bytes of one ia_vote_level call: hit records, pair classes, bounds
size_t vote_level_bytes(const Shape& sh, int32_t n_hits) {
  const int64_t n_tr = int64_t(sh.n_parents) * sh.m012;
  return align_up(sizeof(Persistent)) + align_up(sizeof(HitRec) * size_t(std::max(1, n_hits)) + 1) +
         align_up(size_t(std::max<int64_t>(1, n_tr * int64_t(n_hits))) + 1) + 2 * align_up(4 * size_t(n_tr) + 1);
}

// one level's votes with the context's arena as scratch
ia_status vote_level_run(ia_ctx* c, const ia_hit* d_hits, int32_t n_hits, const uint8_t* d_active,
                         const ia_box* d_parents, const Shape& sh, ia_precision prec, uint16_t* d_votes,
                         void* stream) {
  reset_bump(c);
  HitRec* recs = bump<HitRec>(c, size_t(std::max(1, n_hits)));
  if (!recs) return fail(c, IA_ERR_NOMEM, "scratch too small for %d hits", n_hits);
  hipStream_t s = as_stream(stream);
  Persistent* ps = persistent(c);
  ia::EvView vw = single_view(n_hits);
  if (n_hits > 0)
    hipLaunchKernelGGL(ia::k_prep, dim3((n_hits + 255) / 256, 1), dim3(256), 0, s,
                       reinterpret_cast<const double*>(d_hits), d_active, vw, recs, nullptr, nullptr, nullptr, nullptr,
                       &ps->status,
                       &ps->n_bad, nullptr, nullptr, nullptr, BoxD{}, nullptr, c->vf_xr, c->vf_yr, nullptr);
  // classes of the (triple, hit) pairs and per-triple vote bounds
  const int64_t n_tr = int64_t(sh.n_parents) * sh.m012;
  uint8_t* flags = bump<uint8_t>(c, size_t(std::max<int64_t>(1, n_tr * int64_t(n_hits))));
  int32_t* tlb = bump<int32_t>(c, size_t(n_tr));
  int32_t* tn2 = bump<int32_t>(c, size_t(n_tr));
  if (!flags || !tlb || !tn2)
    return fail(c, IA_ERR_NOMEM, "scratch too small: the level needs %lld bytes of pair classes",
                static_cast<long long>(n_tr * (int64_t(n_hits) + 8)));
  vw.flag_stride = 0;
  vw.tri_stride = 0;
  vw.fwd = c->vf_forward;
  vw.disk = c->vf_disk;
  vw.vref[0] = c->vf_xr;
  vw.vref[1] = c->vf_yr;
  const BoxD* par = reinterpret_cast<const BoxD*>(d_parents);
  const bool f32 = prec == IA_FP32, exact = prec == IA_FP64X, iv = prec == IA_IV;
  const uint32_t fill_n = static_cast<uint32_t>(std::min<int64_t>(n_tr, 0x7fffffff));
  hipLaunchKernelGGL(ia::k_fill_u32, dim3(std::min<uint32_t>((fill_n + 255) / 256, 65535)), dim3(256), 0, s,
                     reinterpret_cast<uint32_t*>(tlb), fill_n, 0u);
  hipLaunchKernelGGL(ia::k_fill_u32, dim3(std::min<uint32_t>((fill_n + 255) / 256, 65535)), dim3(256), 0, s,
                     reinterpret_cast<uint32_t*>(tn2), fill_n, 0u);
  const ia_status cs = launch_classify(c, recs, vw, 1, n_hits, par, sh, flags, tlb, tn2, nullptr, s, f32,
                                       c->slack32, nullptr, nullptr, exact || iv);
  if (cs != IA_OK) return cs;
  if (iv)
    return launch_vote_iv(c, recs, vw, 1, par, sh, flags, d_votes, nullptr, nullptr, tlb, tn2, nullptr, nullptr,
                          nullptr, s);
  const VoteIn in{flags, tlb, tn2, nullptr, 0};
  return launch_vote(c, recs, vw, 1, par, sh, d_votes, nullptr, nullptr, in, nullptr, s, f32, c->slack32, nullptr,
                     exact);
}

}  // namespace

extern "C" {

ia_status ia_vote_level(ia_ctx* c, const ia_hit* d_hits, int32_t n_hits, const uint8_t* d_active,
                        const ia_box* d_parents, int32_t n_parents, const int32_t split[5],
                        ia_precision prec, uint16_t* d_votes, void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (c->pool) return fail(c, IA_ERR_INVALID, "the context holds a resident pool (ia_pool_destroy first)");
  Shape sh;
  const ia_status a = vote_level_args(c, d_hits, n_hits, d_parents, n_parents, split, prec, d_votes, &sh);
  if (a != IA_OK) return a;
  IA_HIP(c, hipSetDevice(c->device));
  return vote_level_run(c, d_hits, n_hits, d_active, d_parents, sh, prec, d_votes, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Scratch of ia_vote_level_noalloc: a fixed array in every device's code
// object, held until the process ends.  Host code uses only the address
// hipGetSymbolAddress returns for the current device, never the array's name.
static __device__ __align__(256) char scratch[IA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
char* g_scratch_at[kMaxDevices] = {};
// this device's copy of `scratch`, looked up once per device (with that
// device current); nullptr when the lookup fails
char* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_at[dev] = static_cast<char*>(p);
  }
  return g_scratch_at[dev];
}

}  // namespace

extern "C" {

ia_status ia_vote_level_noalloc(const ia_hit* d_hits, int32_t n_hits, const uint8_t* d_active,
                                const ia_box* d_parents, int32_t n_parents, const int32_t split[5],
                                ia_precision prec, uint16_t* d_votes, void* stream) {
  // a context on the stack: default settings, the static array as its arena,
  // messages into a per-thread buffer (nothing is allocated)
  ia_ctx c;
  c.errbuf = g_noalloc_err;
  g_noalloc_err[0] = '\0';
  Shape sh;
  const ia_status a = vote_level_args(&c, d_hits, n_hits, d_parents, n_parents, split, prec, d_votes, &sh);
  if (a != IA_OK) return a;
  const size_t need = vote_level_bytes(sh, n_hits);
  if (need > size_t(IA_NOALLOC_SCRATCH_BYTES))
    return fail(&c, IA_ERR_NOMEM, "the level needs %zu bytes of scratch, above the %zu bytes of the fixed array",
                need, size_t(IA_NOALLOC_SCRATCH_BYTES));
  if (int64_t(sh.n_parents) * sh.m012 * int64_t(n_hits) >= (int64_t(1) << 31))
    return fail(&c, IA_ERR_OVERFLOW, "level has 2^31 or more (triple, hit) pairs");
  int dev = 0;
  IA_HIP(&c, hipGetDevice(&dev));
  char* base = scratch_on(dev);
  if (!base) return fail(&c, IA_ERR_DEVICE, "hipGetSymbolAddress of the scratch array failed on device %d", dev);
  c.device = dev;
  c.arena = base;
  c.arena_bytes = IA_NOALLOC_SCRATCH_BYTES;
  // the status words at the start of the array start at zero (a fill kernel,
  // so that the call can be captured in a graph)
  hipStream_t s = as_stream(stream);
  const uint32_t n_words = static_cast<uint32_t>(align_up(sizeof(Persistent)) / 4);
  hipLaunchKernelGGL(ia::k_fill_u32, dim3((n_words + 255) / 256), dim3(256), 0, s,
                     reinterpret_cast<uint32_t*>(base), n_words, 0u);
  IA_HIP(&c, hipGetLastError());
  return vote_level_run(&c, d_hits, n_hits, d_active, d_parents, sh, prec, d_votes, stream);
}

ia_status ia_refine(ia_ctx* c, const ia_box* d_parents, int32_t n_parents, const int32_t split[5],
                    const uint16_t* d_votes, int32_t vote_bound, int32_t top_k, ia_box* d_selected,
                    int64_t* d_selected_index, uint16_t* d_selected_votes, void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (c->pool) return fail(c, IA_ERR_INVALID, "the context holds a resident pool (ia_pool_destroy first)");
  if (!d_parents || !split || !d_votes || !d_selected || !d_selected_index || !d_selected_votes)
    return fail(c, IA_ERR_INVALID, "null pointer argument");
  if (n_parents < 1) return fail(c, IA_ERR_INVALID, "n_parents %d < 1", n_parents);
  if (top_k < 1 || top_k > kMaxTopK) return fail(c, IA_ERR_INVALID, "top_k %d outside [1, %d]", top_k, kMaxTopK);
  if (vote_bound < 0 || vote_bound > 65535) return fail(c, IA_ERR_INVALID, "vote_bound %d", vote_bound);
  Shape sh;
  if (!make_shape(split, n_parents, &sh)) return fail(c, IA_ERR_OVERFLOW, "level exceeds 2^31 - 1 boxes");
  IA_HIP(c, hipSetDevice(c->device));
  reset_bump(c);
  const int32_t n_bins = vote_bound + 1;
  uint32_t chunk;
  const int32_t g = sel_groups(sh.n_boxes, &chunk);
  uint32_t* hist = bump<uint32_t>(c, size_t(n_bins));
  int32_t* cnt = bump<int32_t>(c, 2 * size_t(g));
  uint32_t* tmp = bump<uint32_t>(c, size_t(top_k));
  if (!hist || !cnt || !tmp) return fail(c, IA_ERR_NOMEM, "scratch too small for the selection");
  hipStream_t s = as_stream(stream);
  Persistent* ps = persistent(c);
  hipLaunchKernelGGL(ia::k_fill_u32, dim3((n_bins + 255) / 256), dim3(256), 0, s, hist, uint32_t(n_bins), 0u);
  const uint32_t hg = std::min<uint32_t>((sh.n_boxes + ia::kWG - 1) / ia::kWG, 2048);
  hipLaunchKernelGGL(ia::k_hist, dim3(hg), dim3(ia::kWG), 0, s, d_votes, sh.n_boxes, hist, n_bins, &ps->status);
  return launch_select(c, d_votes, sh, reinterpret_cast<const BoxD*>(d_parents), hist, n_bins, top_k, cnt, tmp,
                       reinterpret_cast<BoxD*>(d_selected), d_selected_index, d_selected_votes, nullptr, 0, s);
}

ia_status ia_estimate(ia_ctx* c, const ia_box* d_parents, int32_t n_parents, const int32_t split[5],
                      const uint16_t* d_votes, ia_estimate_t* d_out, void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (c->pool) return fail(c, IA_ERR_INVALID, "the context holds a resident pool (ia_pool_destroy first)");
  if (!d_parents || !split || !d_votes || !d_out) return fail(c, IA_ERR_INVALID, "null pointer argument");
  if (n_parents < 1) return fail(c, IA_ERR_INVALID, "n_parents %d < 1", n_parents);
  Shape sh;
  if (!make_shape(split, n_parents, &sh)) return fail(c, IA_ERR_OVERFLOW, "level exceeds 2^31 - 1 boxes");
  if (sh.n_boxes > kMaxEstimateBoxes) return fail(c, IA_ERR_OVERFLOW, "level too large for the estimate");
  IA_HIP(c, hipSetDevice(c->device));
  reset_bump(c);
  // the first max-vote box is the rank-0 entry of a top-1 selection
  const int32_t n_bins = 65536;
  uint32_t chunk;
  const int32_t g = sel_groups(sh.n_boxes, &chunk);
  const int32_t n_part = est_parts(sh.n_boxes);
  uint32_t* hist = bump<uint32_t>(c, size_t(n_bins));
  int32_t* cnt = bump<int32_t>(c, 2 * size_t(g));
  uint32_t* tmp = bump<uint32_t>(c, 1);
  BoxD* first = bump<BoxD>(c, 1);
  int64_t* first_idx = bump<int64_t>(c, 1);
  uint16_t* first_v = bump<uint16_t>(c, 1);
  double* part = bump<double>(c, size_t(n_part) * ia::kEstQ);
  if (!hist || !cnt || !tmp || !first || !first_idx || !first_v || !part)
    return fail(c, IA_ERR_NOMEM, "scratch too small for the estimate");
  hipStream_t s = as_stream(stream);
  Persistent* ps = persistent(c);
  const BoxD* par = reinterpret_cast<const BoxD*>(d_parents);
  hipLaunchKernelGGL(ia::k_fill_u32, dim3((n_bins + 255) / 256), dim3(256), 0, s, hist, uint32_t(n_bins), 0u);
  const uint32_t hg = std::min<uint32_t>((sh.n_boxes + ia::kWG - 1) / ia::kWG, 2048);
  hipLaunchKernelGGL(ia::k_hist, dim3(hg), dim3(ia::kWG), 0, s, d_votes, sh.n_boxes, hist, n_bins, &ps->status);
  ia_status st = launch_select(c, d_votes, sh, par, hist, n_bins, 1, cnt, tmp, first, first_idx, first_v, nullptr,
                               0, s);
  if (st != IA_OK) return st;
  ia::EvView vw = single_view(0);
  vw.k = 1;
  vw.part_stride = n_part * ia::kEstQ;
  const uint32_t eper = est_per(n_part, 1);
  hipLaunchKernelGGL(ia::k_est_partial, dim3((n_part + eper - 1) / eper, 1), dim3(ia::kWG), 0, s, par, sh, d_votes,
                     first, first_v, part, vw, nullptr, nullptr, 1, static_cast<uint32_t>(n_part), eper, 0,
                     static_cast<const int32_t*>(nullptr), static_cast<uint32_t*>(nullptr), 0);
  hipLaunchKernelGGL(ia::k_est_final, dim3(1, 1), dim3(ia::kWG), 0, s, part, n_part, first, first_v,
                     reinterpret_cast<ia::EstimateOut*>(d_out), nullptr, nullptr, vw, 0.0, nullptr, nullptr, nullptr,
                     0, static_cast<uint32_t*>(nullptr), 0);
  IA_HIP(c, hipGetLastError());
  return IA_OK;
}

ia_status ia_find_helices(ia_ctx* c, const ia_hit* d_hits, const int32_t* h_off, int32_t n_events,
                          const ia_schedule* sc, ia_helix* d_out, int32_t max_per_event, int32_t* d_n_out,
                          int32_t* d_assigned, void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (c->pool) return fail(c, IA_ERR_INVALID, "the context holds a resident pool (ia_pool_destroy first)");
  if (!h_off || !sc || !d_out || !d_n_out) return fail(c, IA_ERR_INVALID, "null pointer argument");
  if (n_events < 0) return fail(c, IA_ERR_INVALID, "n_events %d < 0", n_events);
  if (max_per_event < 1) return fail(c, IA_ERR_INVALID, "max_per_event %d < 1", max_per_event);
  const ia_status sv = check_sched(c, sc);
  if (sv != IA_OK) return sv;
  const float slack32 = ia::ru32(sc->fp32_slack);
  int32_t max_hits = 0;
  for (int32_t e = 0; e < n_events; ++e) {
    const int32_t n = h_off[e + 1] - h_off[e];
    if (n < 0 || n > kMaxHits) return fail(c, IA_ERR_INVALID, "event %d has %d hits", e, n);
    max_hits = std::max(max_hits, n);
  }
  if (max_hits > 0 && !d_hits) return fail(c, IA_ERR_INVALID, "d_hits is NULL");
  SchedShapes S;
  if (!sched_shapes(sc, &S)) return fail(c, IA_ERR_OVERFLOW, "a level exceeds 2^31 - 1 boxes");
  if (S.max_boxes > kMaxEstimateBoxes)
    return fail(c, IA_ERR_OVERFLOW, "a level exceeds %lld boxes", static_cast<long long>(kMaxEstimateBoxes));
  IA_HIP(c, hipSetDevice(c->device));
  const int32_t K = sched_k(sc);
  // events per chunk: as many as the arena holds.  Staged records: room for
  // every (triple, hit) pair when a full chunk fits that way, else kRecCap
  // per event (an event needing more is voted with in-kernel staging)
  const int64_t worst_rec = std::max<int64_t>(1, S.max_triples * int64_t(max_hits));
  auto chunk_for = [&](int64_t rpe, int32_t* out) {
    FindLayout L1, L2;
    layout_find(S.max_boxes, S.max_triples, K, max_hits, 1, max_hits, &L1, rpe);
    if (L1.total > c->arena_bytes) return false;
    layout_find(S.max_boxes, S.max_triples, K, max_hits, 2, 2 * int64_t(max_hits), &L2, rpe);
    const size_t per_event = L2.total - L1.total;
    int32_t ch = static_cast<int32_t>(std::min<size_t>(
        std::max(1, n_events), 1 + (c->arena_bytes - L1.total) / std::max<size_t>(per_event, 1)));
    *out = std::max(1, std::min(ch, std::min(c->max_chunk, 65535)));
    return true;
  };
  const int32_t want = std::max(1, std::min(n_events, std::min(c->max_chunk, 65535)));
  int64_t rpe = worst_rec;
  int32_t chunk = 0;
  const bool fits_worst = chunk_for(rpe, &chunk);
  if ((!fits_worst || chunk < want) && kRecCap < worst_rec) {
    int32_t chunk_cap = 0;
    if (chunk_for(kRecCap, &chunk_cap) && (!fits_worst || chunk_cap > chunk)) {
      rpe = kRecCap;
      chunk = chunk_cap;
      // as many records per event as the arena holds at that chunk size
      // (fewer events fall back to the in-kernel staging)
      for (int64_t r = 2 * kRecCap; r < worst_rec; r *= 2) {
        int32_t ch2 = 0;
        if (!chunk_for(r, &ch2) || ch2 < chunk) break;
        rpe = r;
      }
    }
  }
  if (chunk == 0) {
    FindLayout L1;
    layout_find(S.max_boxes, S.max_triples, K, max_hits, 1, max_hits, &L1, rpe);
    return fail(c, IA_ERR_NOMEM, "scratch too small: need %zu bytes, have %zu", L1.total, c->arena_bytes);
  }
  const bool may_overflow = rpe < worst_rec;
  hipStream_t s = as_stream(stream);
  chunk = std::min(chunk, kOffSlotInts - 1);
  for (int32_t e0 = 0; e0 < n_events; e0 += chunk) {
    const int32_t E = std::min(chunk, n_events - e0);
    int32_t cmax = 0;
    for (int32_t e = e0; e < e0 + E; ++e) cmax = std::max(cmax, h_off[e + 1] - h_off[e]);
    const int64_t n_tot = int64_t(h_off[e0 + E]) - h_off[e0];
    const ia_status st = run_chunk(c, reinterpret_cast<const double*>(d_hits) + 8 * int64_t(h_off[e0]), h_off + e0,
                                   nullptr, E, cmax, n_tot, S, sc, slack32, rpe, may_overflow,
                                   reinterpret_cast<ia::HelixOut*>(d_out) + int64_t(e0) * max_per_event,
                                   max_per_event, d_n_out + e0, d_assigned ? d_assigned + h_off[e0] : nullptr, s);
    if (st != IA_OK) return st;
  }
  return IA_OK;
}

ia_status ia_ctx_autotune(ia_ctx* c, const ia_hit* d_hits, const int32_t* h_off, int32_t n_events,
                          const ia_schedule* sc, ia_helix* d_out, int32_t max_per_event, int32_t* d_n_out,
                          void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (c->pool) return fail(c, IA_ERR_INVALID, "the context holds a resident pool (ia_pool_destroy first)");
  static const int32_t kTiles[3] = {256, 128, 64};
  const int32_t saved = c->tile_override;
  const bool saved_prof = c->profiling;
  // summed vote-kernel milliseconds per (level size, candidate)
  std::vector<std::pair<uint32_t, double>> ms[3];
  for (int ci = 0; ci < 3; ++ci) {
    c->tile_override = kTiles[ci];
    c->profiling = false;
    ia_status st = ia_find_helices(c, d_hits, h_off, n_events, sc, d_out, max_per_event, d_n_out, nullptr, stream);
    if (st == IA_OK) {
      c->profiling = true;
      st = ia_find_helices(c, d_hits, h_off, n_events, sc, d_out, max_per_event, d_n_out, nullptr, stream);
    }
    c->profiling = false;
    if (st == IA_OK) IA_HIP(c, hipStreamSynchronize(as_stream(stream)));
    for (auto& m : c->marks) {
      float t = 0.f;
      if (st == IA_OK && m.kind == IA_KERNEL_VOTE && hipEventElapsedTime(&t, m.e0, m.e1) == hipSuccess) {
        bool found = false;
        for (auto& x : ms[ci])
          if (x.first == m.n_boxes) { x.second += t; found = true; }
        if (!found) ms[ci].push_back({m.n_boxes, double(t)});
      }
      (void)hipEventDestroy(m.e0);
      (void)hipEventDestroy(m.e1);
    }
    c->marks.clear();
    if (st != IA_OK) {
      c->tile_override = saved;
      c->profiling = saved_prof;
      return st;
    }
  }
  c->tile_override = saved;
  c->profiling = saved_prof;
  c->tuned.clear();
  for (const auto& x : ms[0]) {
    int32_t best = kTiles[0];
    double best_ms = x.second;
    for (int ci = 1; ci < 3; ++ci)
      for (const auto& y : ms[ci])
        if (y.first == x.first && y.second < best_ms) { best_ms = y.second; best = kTiles[ci]; }
    c->tuned.push_back({x.first, best});
  }
  return IA_OK;
}

int32_t ia_ctx_tuned(const ia_ctx* c, uint32_t* n_boxes, int32_t* tiles, int32_t max_entries) {
  if (!c) return 0;
  const int32_t n = static_cast<int32_t>(c->tuned.size());
  for (int32_t i = 0; i < n && i < max_entries; ++i) {
    if (n_boxes) n_boxes[i] = c->tuned[i].first;
    if (tiles) tiles[i] = c->tuned[i].second;
  }
  return n;
}

ia_status ia_find_helices_dev(ia_ctx* c, const ia_hit* d_hits, const int32_t* d_off, int32_t n_events,
                              int32_t max_hits, int64_t n_hits_total, const ia_schedule* sc, ia_helix* d_out,
                              int32_t max_per_event, int32_t* d_n_out, int32_t* d_assigned, void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (c->pool) return fail(c, IA_ERR_INVALID, "the context holds a resident pool (ia_pool_destroy first)");
  if (!d_off || !sc || !d_out || !d_n_out) return fail(c, IA_ERR_INVALID, "null pointer argument");
  if (n_events < 1 || n_events > 65535) return fail(c, IA_ERR_INVALID, "n_events %d outside [1, 65535]", n_events);
  if (max_per_event < 1) return fail(c, IA_ERR_INVALID, "max_per_event %d < 1", max_per_event);
  if (max_hits < 1 || max_hits > kMaxHits) return fail(c, IA_ERR_INVALID, "max_hits %d outside [1, %d]", max_hits, kMaxHits);
  if (n_hits_total < 0) return fail(c, IA_ERR_INVALID, "n_hits_total < 0");
  if (n_hits_total > 0 && !d_hits) return fail(c, IA_ERR_INVALID, "d_hits is NULL");
  const ia_status sv = check_sched(c, sc);
  if (sv != IA_OK) return sv;
  const float slack32 = ia::ru32(sc->fp32_slack);
  SchedShapes S;
  if (!sched_shapes(sc, &S)) return fail(c, IA_ERR_OVERFLOW, "a level exceeds 2^31 - 1 boxes");
  if (S.max_boxes > kMaxEstimateBoxes)
    return fail(c, IA_ERR_OVERFLOW, "a level exceeds %lld boxes", static_cast<long long>(kMaxEstimateBoxes));
  IA_HIP(c, hipSetDevice(c->device));
  // records for every (triple, hit) pair when they fit, else kRecCap per event
  const int64_t worst_rec = std::max<int64_t>(1, S.max_triples * int64_t(max_hits));
  int64_t rpe = worst_rec;
  FindLayout L;
  layout_find(S.max_boxes, S.max_triples, sched_k(sc), max_hits, n_events, n_hits_total, &L, rpe);
  if (L.total > c->arena_bytes && kRecCap < worst_rec) {
    rpe = kRecCap;
    layout_find(S.max_boxes, S.max_triples, sched_k(sc), max_hits, n_events, n_hits_total, &L, rpe);
    // as many records per event as the arena holds
    for (int64_t r = 2 * kRecCap; r < worst_rec; r *= 2) {
      FindLayout L2;
      layout_find(S.max_boxes, S.max_triples, sched_k(sc), max_hits, n_events, n_hits_total, &L2, r);
      if (L2.total > c->arena_bytes) break;
      rpe = r;
      L = L2;
    }
  }
  if (L.total > c->arena_bytes)
    return fail(c, IA_ERR_NOMEM, "scratch too small: need %zu bytes, have %zu", L.total, c->arena_bytes);
  return run_chunk(c, reinterpret_cast<const double*>(d_hits), nullptr, d_off, n_events, max_hits, n_hits_total, S, sc,
                   slack32, rpe, rpe < worst_rec, reinterpret_cast<ia::HelixOut*>(d_out), max_per_event, d_n_out,
                   d_assigned, as_stream(stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Resident pools: continuous batching at helix-pass granularity.  The pool
// lays out the whole search state of `rows` events of up to max_hits hits in
// the context's arena (the layout ia_find_helices uses for a chunk of that
// many events, plus a hit store of fixed-size rows).  Admission copies a new
// event's hits into a free row and prepares that row alone; a step runs one
// helix pass (every level of the window schedule) over all rows still
// searching, so events admitted at different times share the launches.
struct PoolState {
  int32_t rows = 0, max_hits = 0, max_out = 0;
  ia_schedule sc{};
  SchedShapes S{};
  FindLayout L{};
  int64_t rpe = 0;
  bool may_overflow = false;
  float slack32 = 0.f;
  size_t store = 0, cnt = 0, newrows = 0, newoff = 0, out = 0, n_out = 0, assigned = 0, state = 0, total = 0;
};

namespace {

// the pool's extra arrays after the find layout; false when it does not fit
bool pool_layout(PoolState* P, size_t arena_bytes) {
  layout_find(P->S.max_boxes, P->S.max_triples, sched_k(&P->sc), P->max_hits, P->rows,
              int64_t(P->rows) * P->max_hits, &P->L, P->rpe);
  size_t off = align_up(P->L.total);
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes + 1);
    return o;
  };
  const size_t R = size_t(P->rows), H = size_t(P->max_hits);
  P->store = take(sizeof(double) * 8 * R * H);
  P->cnt = take(sizeof(int32_t) * R);
  P->newrows = take(sizeof(int32_t) * R);
  P->newoff = take(sizeof(int32_t) * (R + 1));
  P->out = take(sizeof(ia::HelixOut) * R * size_t(P->max_out));
  P->n_out = take(sizeof(int32_t) * R);
  P->assigned = take(sizeof(int32_t) * R * H);
  P->state = take(sizeof(int32_t) * 2 * R);
  P->total = off;
  return P->total <= arena_bytes;
}

// records per event: every (triple, hit) pair when the pool fits that way,
// else the most (doubling from kRecCap) that fit; false when none fits
bool pool_fit(PoolState* P, size_t arena_bytes) {
  const int64_t worst = std::max<int64_t>(1, P->S.max_triples * int64_t(P->max_hits));
  P->rpe = worst;
  if (pool_layout(P, arena_bytes)) {
    P->may_overflow = false;
    return true;
  }
  if (kRecCap >= worst) return false;
  P->rpe = kRecCap;
  if (!pool_layout(P, arena_bytes)) return false;
  for (int64_t r = 2 * kRecCap; r < worst; r *= 2) {
    PoolState Q = *P;
    Q.rpe = r;
    if (!pool_layout(&Q, arena_bytes)) break;
    *P = Q;
  }
  P->may_overflow = true;
  return true;
}

ia::EvView pool_view(ia_ctx* c, const PoolState* P) {
  char* a = c->arena;
  const FindLayout& L = P->L;
  ia::EvView vw{};
  vw.off = reinterpret_cast<const int32_t*>(a + L.off);
  vw.cnt = reinterpret_cast<const int32_t*>(a + P->cnt);
  vw.k = sched_k(&P->sc);
  vw.flag_stride = L.flag_stride;
  vw.tri_stride = L.tri_stride;
  vw.rec_stride = L.rec_stride;
  vw.pflag_stride = L.pflag_stride;
  vw.hist_stride = L.hist_stride;
  vw.wg_stride = L.wg_stride;
  vw.part_stride = L.part_stride;
  vw.max_out = P->max_out;
  vw.max_hits = P->max_hits;
  vw.n_total = int64_t(P->rows) * P->max_hits;
  vw.disk = P->sc.disk;
  return vw;
}

}  // namespace

extern "C" {

int32_t ia_pool_capacity(const ia_ctx* c, int32_t max_hits, const ia_schedule* sc, int32_t max_per_event) {
  if (!c || !sc || max_hits < 1 || max_hits > kMaxHits || max_per_event < 1) return 0;
  PoolState P;
  P.max_hits = max_hits;
  P.sc = *sc;
  P.max_out = std::min(sc->n_helix_max, max_per_event);
  if (P.max_out < 1 || !sched_shapes(sc, &P.S)) return 0;
  int32_t lo = 0, hi = 65535;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) / 2;
    P.rows = mid;
    if (pool_fit(&P, c->arena_bytes)) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

ia_status ia_pool_create(ia_ctx* c, int32_t rows, int32_t max_hits, const ia_schedule* sc, int32_t max_per_event,
                         void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (c->pool) return fail(c, IA_ERR_INVALID, "the context already holds a pool");
  if (!sc) return fail(c, IA_ERR_INVALID, "null schedule");
  if (rows < 1 || rows > 65535) return fail(c, IA_ERR_INVALID, "rows %d outside [1, 65535]", rows);
  if (max_hits < 1 || max_hits > kMaxHits) return fail(c, IA_ERR_INVALID, "max_hits %d outside [1, %d]", max_hits, kMaxHits);
  if (max_per_event < 1) return fail(c, IA_ERR_INVALID, "max_per_event %d < 1", max_per_event);
  const ia_status sv = check_sched(c, sc);
  if (sv != IA_OK) return sv;
  if (sc->mode != IA_SCHED_WINDOW) return fail(c, IA_ERR_INVALID, "pools run the window schedule only");
  IA_HIP(c, hipSetDevice(c->device));
  PoolState* P = new PoolState();
  P->rows = rows;
  P->max_hits = max_hits;
  P->sc = *sc;
  P->max_out = std::min(sc->n_helix_max, max_per_event);
  P->slack32 = ia::ru32(sc->fp32_slack);
  if (!sched_shapes(sc, &P->S) || P->S.max_boxes > kMaxEstimateBoxes) {
    delete P;
    return fail(c, IA_ERR_OVERFLOW, "a level of the schedule is too large");
  }
  if (!pool_fit(P, c->arena_bytes)) {
    const size_t need = P->total;
    delete P;
    return fail(c, IA_ERR_NOMEM, "scratch too small for the pool: need %zu bytes, have %zu", need, c->arena_bytes);
  }
  char* a = c->arena;
  BoxD rb;
  std::memcpy(&rb, &sc->range, sizeof rb);
  hipLaunchKernelGGL(ia::k_pool_init, dim3(std::max(1, std::min(1024, (rows + 256) / 256))), dim3(256), 0,
                     as_stream(stream), reinterpret_cast<int32_t*>(a + P->L.off), reinterpret_cast<int32_t*>(a + P->cnt),
                     reinterpret_cast<EventState*>(a + P->L.ev), reinterpret_cast<int32_t*>(a + P->n_out), rows,
                     max_hits, reinterpret_cast<BoxD*>(a + P->L.range), rb);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    delete P;
    return fail(c, IA_ERR_DEVICE, "k_pool_init: %s", hipGetErrorString(e));
  }
  c->pool = P;
  return IA_OK;
}

ia_status ia_pool_destroy(ia_ctx* c) {
  if (!c) return IA_ERR_INVALID;
  delete c->pool;
  c->pool = nullptr;
  return IA_OK;
}

ia_status ia_pool_admit(ia_ctx* c, int32_t n, const int32_t* h_rows, const ia_hit* d_hits, const int32_t* h_off,
                        void* stream) {
  if (!c) return IA_ERR_INVALID;
  PoolState* P = c->pool;
  if (!P) return fail(c, IA_ERR_INVALID, "no pool on this context");
  if (n == 0) return IA_OK;
  if (n < 0 || n > P->rows || 2 * n + 1 > kOffSlotInts)
    return fail(c, IA_ERR_INVALID, "%d events outside [0, %d]", n, std::min(P->rows, (kOffSlotInts - 1) / 2));
  if (!h_rows || !h_off) return fail(c, IA_ERR_INVALID, "null pointer argument");
  std::vector<char> seen(size_t(P->rows), 0);
  for (int32_t j = 0; j < n; ++j) {
    const int32_t r = h_rows[j], k = h_off[j + 1] - h_off[j];
    if (r < 0 || r >= P->rows) return fail(c, IA_ERR_INVALID, "row %d outside [0, %d)", r, P->rows);
    if (seen[size_t(r)]) return fail(c, IA_ERR_INVALID, "row %d admitted twice", r);
    seen[size_t(r)] = 1;
    if (k < 0 || k > P->max_hits) return fail(c, IA_ERR_INVALID, "event %d has %d hits (rows hold %d)", j, k, P->max_hits);
  }
  if (h_off[n] > h_off[0] && !d_hits) return fail(c, IA_ERR_INVALID, "d_hits is NULL");
  IA_HIP(c, hipSetDevice(c->device));
  hipStream_t s = as_stream(stream);
  char* a = c->arena;
  // rows and event-relative offsets through a pinned slot whose last copy is done
  const uint32_t slot = c->slot_next++ % kOffSlots;
  if (c->slot_used[slot]) IA_HIP(c, hipEventSynchronize(c->slot_done[slot]));
  int32_t* ho = c->pinned + size_t(slot) * kOffSlotInts;
  for (int32_t j = 0; j < n; ++j) ho[j] = h_rows[j];
  for (int32_t j = 0; j <= n; ++j) ho[n + j] = h_off[j] - h_off[0];
  int32_t* d_rows = reinterpret_cast<int32_t*>(a + P->newrows);
  int32_t* d_noff = reinterpret_cast<int32_t*>(a + P->newoff);
  IA_HIP(c, hipMemcpyAsync(d_rows, ho, sizeof(int32_t) * size_t(n), hipMemcpyHostToDevice, s));
  IA_HIP(c, hipMemcpyAsync(d_noff, ho + n, sizeof(int32_t) * (size_t(n) + 1), hipMemcpyHostToDevice, s));
  IA_HIP(c, hipEventRecord(c->slot_done[slot], s));
  c->slot_used[slot] = true;
  const double* src = reinterpret_cast<const double*>(d_hits) + 8 * int64_t(h_off[0]);
  double* store = reinterpret_cast<double*>(a + P->store);
  const int32_t gx = std::max(1, std::min(64, (P->max_hits * 8 + 255) / 256));
  hipLaunchKernelGGL(ia::k_pool_load, dim3(gx, n), dim3(256), 0, s, src, d_noff, d_rows, store,
                     reinterpret_cast<int32_t*>(a + P->cnt), P->max_hits);
  // prepare the new rows alone: state, counters, prepared hits, assignments
  const FindLayout& L = P->L;
  Persistent* ps = persistent(c);
  const ia::EvView vw = pool_view(c, P);
  const int32_t pg = std::max(1, (P->max_hits + 2 + 255) / 256);
  hipLaunchKernelGGL(ia::k_prep, dim3(pg, n), dim3(256), 0, s, store, nullptr, vw,
                     reinterpret_cast<HitRec*>(a + L.recs), reinterpret_cast<uint32_t*>(a + L.hist),
                     reinterpret_cast<uint32_t*>(a + L.lbh), reinterpret_cast<int32_t*>(a + L.tlb),
                     reinterpret_cast<int32_t*>(a + L.tn2), &ps->status, &ps->n_bad,
                     reinterpret_cast<EventState*>(a + L.ev), reinterpret_cast<int32_t*>(a + P->n_out),
                     static_cast<BoxD*>(nullptr), BoxD{}, reinterpret_cast<int32_t*>(a + P->assigned), 0.0, 0.0,
                     d_rows);
  IA_HIP(c, hipGetLastError());
  return IA_OK;
}

ia_status ia_pool_step(ia_ctx* c, void* stream) {
  if (!c) return IA_ERR_INVALID;
  PoolState* P = c->pool;
  if (!P) return fail(c, IA_ERR_INVALID, "no pool on this context");
  IA_HIP(c, hipSetDevice(c->device));
  char* a = c->arena;
  const FindLayout& L = P->L;
  const RecIn rin{reinterpret_cast<int32_t*>(a + L.live_tri), reinterpret_cast<int32_t*>(a + L.rec_off),
                  reinterpret_cast<int32_t*>(a + L.rec_fill), a + L.rec,
                  reinterpret_cast<ia::TriFrame*>(a + L.tfr), reinterpret_cast<int32_t*>(a + L.live_off),
                  reinterpret_cast<int64_t*>(a + L.stage_off)};
  // one pass, numbered as a later pass: it starts by taking every row back
  // to the origin's frame with all its remaining hits (a no-op for a row
  // just admitted)
  return run_window(c, reinterpret_cast<const double*>(a + P->store), pool_view(c, P), P->rows, P->max_hits, P->S,
                    &P->sc, P->slack32, P->may_overflow, L, reinterpret_cast<HitRec*>(a + L.recs),
                    reinterpret_cast<uint16_t*>(a + L.votes), reinterpret_cast<uint32_t*>(a + L.hist),
                    reinterpret_cast<BoxD*>(a + L.selA), reinterpret_cast<BoxD*>(a + L.range),
                    reinterpret_cast<int64_t*>(a + L.sel_idx), reinterpret_cast<uint16_t*>(a + L.sel_v),
                    reinterpret_cast<EventState*>(a + L.ev), reinterpret_cast<double*>(a + L.part),
                    reinterpret_cast<uint8_t*>(a + L.flags), reinterpret_cast<uint8_t*>(a + L.pflags),
                    reinterpret_cast<ia::ParentE*>(a + L.pe), reinterpret_cast<int32_t*>(a + L.tlb),
                    reinterpret_cast<int32_t*>(a + L.tn2), reinterpret_cast<uint32_t*>(a + L.lbh),
                    reinterpret_cast<int32_t*>(a + L.wg_max), reinterpret_cast<int32_t*>(a + L.live), rin,
                    reinterpret_cast<int32_t*>(a + P->assigned), reinterpret_cast<ia::HelixOut*>(a + P->out),
                    reinterpret_cast<int32_t*>(a + P->n_out), 1, 2, as_stream(stream));
}

ia_status ia_pool_poll(ia_ctx* c, int32_t* h_state, void* stream) {
  if (!c) return IA_ERR_INVALID;
  PoolState* P = c->pool;
  if (!P) return fail(c, IA_ERR_INVALID, "no pool on this context");
  if (!h_state) return fail(c, IA_ERR_INVALID, "null pointer argument");
  IA_HIP(c, hipSetDevice(c->device));
  hipStream_t s = as_stream(stream);
  char* a = c->arena;
  int32_t* d_state = reinterpret_cast<int32_t*>(a + P->state);
  hipLaunchKernelGGL(ia::k_pool_state, dim3(std::max(1, std::min(256, (P->rows + 255) / 256))), dim3(256), 0, s,
                     reinterpret_cast<const EventState*>(a + P->L.ev), reinterpret_cast<const int32_t*>(a + P->n_out),
                     P->rows, d_state);
  IA_HIP(c, hipGetLastError());
  IA_HIP(c, hipMemcpyAsync(h_state, d_state, sizeof(int32_t) * 2 * size_t(P->rows), hipMemcpyDeviceToHost, s));
  IA_HIP(c, hipStreamSynchronize(s));
  return IA_OK;
}

ia_status ia_pool_take(ia_ctx* c, int32_t row, int32_t n_helices, ia_helix* h_out, int32_t n_hits,
                       int32_t* h_assigned, void* stream) {
  if (!c) return IA_ERR_INVALID;
  PoolState* P = c->pool;
  if (!P) return fail(c, IA_ERR_INVALID, "no pool on this context");
  if (row < 0 || row >= P->rows) return fail(c, IA_ERR_INVALID, "row %d outside [0, %d)", row, P->rows);
  if (n_helices < 0 || n_helices > P->max_out || n_hits < 0 || n_hits > P->max_hits)
    return fail(c, IA_ERR_INVALID, "%d helices / %d hits outside the row", n_helices, n_hits);
  if ((n_helices && !h_out) || (n_hits && !h_assigned)) return fail(c, IA_ERR_INVALID, "null pointer argument");
  IA_HIP(c, hipSetDevice(c->device));
  hipStream_t s = as_stream(stream);
  char* a = c->arena;
  if (n_helices)
    IA_HIP(c, hipMemcpyAsync(h_out, a + P->out + sizeof(ia::HelixOut) * size_t(row) * P->max_out,
                             sizeof(ia::HelixOut) * size_t(n_helices), hipMemcpyDeviceToHost, s));
  if (n_hits)
    IA_HIP(c, hipMemcpyAsync(h_assigned, a + P->assigned + sizeof(int32_t) * size_t(row) * P->max_hits,
                             sizeof(int32_t) * size_t(n_hits), hipMemcpyDeviceToHost, s));
  IA_HIP(c, hipStreamSynchronize(s));
  return IA_OK;
}

}  // extern "C"
