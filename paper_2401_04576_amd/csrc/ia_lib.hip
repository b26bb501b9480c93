// ia_lib.hip -- host side of libia: context, argument checks, launches.
// The C ABI is declared in include/ia.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
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
static_assert(sizeof(HitRec) == 96, "HitRec layout");

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kMaxHits = 65535;
constexpr int32_t kMaxTopK = ia::kMaxTopK;
constexpr int64_t kMaxLevelBoxes = (int64_t(1) << 31) - 1;
constexpr int64_t kSelChunkMin = 4096;
constexpr int32_t kSelMaxGroups = 1024;
// k_estimate: 256 lanes x segments of at most 2^(kEstLevels - 1) boxes
constexpr int64_t kMaxEstimateBoxes = int64_t(ia::kWG) << (ia::kEstLevels - 1);

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Persistent {        // fixed region at the start of the arena
  uint32_t status;
  uint32_t done_counter;
  int64_t n_bad;
};

}  // namespace

struct ia_ctx {
  int32_t device = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  size_t used = 0;
  std::string err;
  bool profiling = false;
  int32_t tile_override = 0;
  int32_t filter_mode = -1;       // -1: automatic, 0: off, 1: on
  std::vector<std::pair<hipEvent_t, hipEvent_t>> marks;
};

namespace {

ia_status fail(ia_ctx* c, ia_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
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

// boxes per workgroup of the vote kernel for a level: large levels use one
// lane per box; small levels split each chunk's hits over 2 or 4 waves so
// that the device gets enough workgroups
int32_t vote_tile(const ia_ctx* c, uint32_t n_boxes) {
  if (c->tile_override) return c->tile_override;
  if (n_boxes >= (1u << 19)) return 256;
  return 128;
}

// the (triple, hit) pre-pass pays when many boxes share a triple
int32_t use_filter(const ia_ctx* c, const Shape& sh) {
  if (c->filter_mode >= 0) return c->filter_mode;
  return sh.m34 >= 64 ? 1 : 0;
}

// launches the (triple, hit) pre-pass when it pays and room allows; returns
// the flags to hand to the vote kernel, or nullptr
const uint8_t* launch_filter(ia_ctx* c, const HitRec* recs, int32_t n, const BoxD* par, const Shape& sh,
                             uint8_t* flags, size_t flag_cap, EventState* ev, hipStream_t s) {
  if (!flags || n <= 0 || !use_filter(c, sh)) return nullptr;
  const uint64_t pairs = uint64_t(sh.n_parents) * sh.m012 * uint64_t(n);
  if (pairs > flag_cap || pairs >= (uint64_t(1) << 31)) return nullptr;
  const uint32_t grid = static_cast<uint32_t>((pairs + ia::kWG - 1) / ia::kWG);
  hipLaunchKernelGGL(ia::k_pair_filter, dim3(grid), dim3(ia::kWG), 0, s, recs, n, par, sh, flags, 1, ev);
  return flags;
}

// launches the vote kernel (with the fused selection when sel.k > 0),
// bracketed by events when profiling
ia_status launch_vote(ia_ctx* c, const HitRec* recs, int32_t n, const BoxD* par, const Shape& sh, uint16_t* votes,
                      uint32_t* hist, int32_t n_bins, const EventState* ev, const uint8_t* flags, int32_t* wg_max,
                      hipStream_t s, int32_t* tile_used = nullptr) {
  const int32_t bx = vote_tile(c, sh.n_boxes);
  const uint32_t grid = (sh.n_boxes + bx - 1) / bx;
  if (tile_used) *tile_used = bx;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profiling) {
    IA_HIP(c, hipEventCreate(&e0));
    IA_HIP(c, hipEventCreate(&e1));
    IA_HIP(c, hipEventRecord(e0, s));
  }
  uint32_t* st = &persistent(c)->status;
  switch (bx) {
    case 256:
      hipLaunchKernelGGL(ia::k_vote<256>, dim3(grid), dim3(ia::kWG), 0, s, recs, n, par, sh, votes, hist, n_bins, st, ev,
                         flags, wg_max);
      break;
    case 128:
      hipLaunchKernelGGL(ia::k_vote<128>, dim3(grid), dim3(ia::kWG), 0, s, recs, n, par, sh, votes, hist, n_bins, st, ev,
                         flags, wg_max);
      break;
    default:
      hipLaunchKernelGGL(ia::k_vote<64>, dim3(grid), dim3(ia::kWG), 0, s, recs, n, par, sh, votes, hist, n_bins, st, ev,
                         flags, wg_max);
      break;
  }
  if (c->profiling) {
    IA_HIP(c, hipEventRecord(e1, s));
    c->marks.emplace_back(e0, e1);
  }
  IA_HIP(c, hipGetLastError());
  return IA_OK;
}

// estimate of a level from its selection (rank 0 = first max-vote box)
ia_status launch_estimate(ia_ctx* c, const BoxD* par, const Shape& sh, const uint16_t* votes, const BoxD* first_box,
                          const uint16_t* first_votes, double* part, ia::EstimateOut* out, EventState* ev,
                          HitRec* recs, int32_t n_hits, double scale, int32_t* assigned, ia::HelixOut* hout,
                          int32_t max_out, int32_t* n_out, hipStream_t s) {
  const int32_t n_part = est_parts(sh.n_boxes);
  hipLaunchKernelGGL(ia::k_est_partial, dim3(n_part), dim3(ia::kWG), 0, s, par, sh, votes, first_box, first_votes,
                     part, ev);
  hipLaunchKernelGGL(ia::k_est_final, dim3(1), dim3(ia::kWG), 0, s, part, n_part, first_box, first_votes, out, ev,
                     recs, n_hits, scale, assigned, hout, max_out, n_out);
  IA_HIP(c, hipGetLastError());
  return IA_OK;
}

// scratch layout of ia_find_helices (byte offsets into the arena)
struct FindLayout {
  size_t recs, votes, hist, cnt, tmp, selA, selB, range, sel_idx, sel_v, ev, part, flags, wg_max, total;
  size_t flag_cap;
};

void layout_find(int64_t max_level_boxes, int64_t max_triples, int32_t top_k, int32_t max_hits, FindLayout* L) {
  uint32_t chunk;
  const int32_t g = sel_groups(max_level_boxes, &chunk);
  const int32_t n_part = est_parts(static_cast<uint32_t>(max_level_boxes));
  size_t off = align_up(sizeof(Persistent));
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes + 1);
    return o;
  };
  L->recs = take(sizeof(HitRec) * size_t(std::max(1, max_hits)));
  L->votes = take(sizeof(uint16_t) * size_t(max_level_boxes));
  L->hist = take(sizeof(uint32_t) * size_t(max_hits + 2));
  L->cnt = take(sizeof(int32_t) * 2 * size_t(g));
  L->tmp = take(sizeof(uint32_t) * size_t(top_k));
  L->selA = take(sizeof(BoxD) * size_t(top_k));
  L->selB = take(sizeof(BoxD) * size_t(top_k));
  L->range = take(sizeof(BoxD));
  L->sel_idx = take(sizeof(int64_t) * size_t(top_k));
  L->sel_v = take(sizeof(uint16_t) * size_t(top_k));
  L->ev = take(sizeof(EventState));
  L->part = take(sizeof(double) * ia::kEstQ * size_t(n_part));
  L->flag_cap = size_t(max_triples) * size_t(std::max(0, max_hits));
  L->flags = take(L->flag_cap);
  L->wg_max = take(sizeof(int32_t) * size_t((max_level_boxes + 63) / 64));
  L->total = off;
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
  reset_bump(c);
  *out = c;
  return IA_OK;
}

void ia_ctx_destroy(ia_ctx* c) {
  if (!c) return;
  for (auto& m : c->marks) {
    (void)hipEventDestroy(m.first);
    (void)hipEventDestroy(m.second);
  }
  if (c->arena) {
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->arena);
  }
  delete c;
}

const char* ia_last_error(const ia_ctx* c) { return c ? c->err.c_str() : "null context"; }

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

ia_status ia_ctx_set_prefilter(ia_ctx* c, int32_t mode) {
  if (!c) return IA_ERR_INVALID;
  if (mode < -1 || mode > 1) return fail(c, IA_ERR_INVALID, "prefilter mode %d not in {-1, 0, 1}", mode);
  c->filter_mode = mode;
  return IA_OK;
}

ia_status ia_ctx_set_profiling(ia_ctx* c, int32_t enable) {
  if (!c) return IA_ERR_INVALID;
  c->profiling = enable != 0;
  return IA_OK;
}

ia_status ia_ctx_profile_read(ia_ctx* c, int64_t* n_launches, double* total_ms) {
  if (!c) return IA_ERR_INVALID;
  IA_HIP(c, hipSetDevice(c->device));
  double tot = 0.0;
  int64_t n = 0;
  ia_status st = IA_OK;
  for (auto& m : c->marks) {
    if (st == IA_OK) {
      hipError_t e = hipEventSynchronize(m.second);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.first, m.second);
      if (e != hipSuccess) st = fail(c, IA_ERR_DEVICE, "profile events: %s", hipGetErrorString(e));
      tot += ms;
      ++n;
    }
    (void)hipEventDestroy(m.first);
    (void)hipEventDestroy(m.second);
  }
  c->marks.clear();
  if (n_launches) *n_launches = n;
  if (total_ms) *total_ms = tot;
  return st;
}

size_t ia_ctx_scratch_needed(const ia_schedule* sc, int32_t max_hits) {
  if (!sc || max_hits < 0) return 0;
  int64_t nb0 = 1, nc = 1;
  for (int j = 0; j < 5; ++j) { nb0 *= std::max(1, sc->bins[j]); nc *= std::max(1, sc->split[j]); }
  const int64_t nbr = int64_t(std::max(1, sc->top_k)) * nc;
  const int64_t nb = std::min<int64_t>(std::max(nb0, nbr), kMaxLevelBoxes);
  const int64_t nt0 = int64_t(std::max(1, sc->bins[0])) * std::max(1, sc->bins[1]) * std::max(1, sc->bins[2]);
  const int64_t ntr = int64_t(std::max(1, sc->top_k)) * std::max(1, sc->split[0]) * std::max(1, sc->split[1]) *
                      std::max(1, sc->split[2]);
  FindLayout L;
  layout_find(nb, std::max(nt0, ntr), std::max(1, sc->top_k), max_hits, &L);
  return L.total;
}

ia_status ia_vote_level(ia_ctx* c, const ia_hit* d_hits, int32_t n_hits, const uint8_t* d_active,
                        const ia_box* d_parents, int32_t n_parents, const int32_t split[5],
                        ia_precision prec, uint16_t* d_votes, void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (n_hits < 0 || n_hits > kMaxHits) return fail(c, IA_ERR_INVALID, "n_hits %d outside [0, %d]", n_hits, kMaxHits);
  if (n_hits > 0 && !d_hits) return fail(c, IA_ERR_INVALID, "d_hits is NULL");
  if (!d_parents || !split || !d_votes) return fail(c, IA_ERR_INVALID, "null pointer argument");
  if (n_parents < 1) return fail(c, IA_ERR_INVALID, "n_parents %d < 1", n_parents);
  if (prec != IA_FP64) return fail(c, IA_ERR_UNSUPPORTED, "precision %d not available", int(prec));
  Shape sh;
  if (!make_shape(split, n_parents, &sh)) return fail(c, IA_ERR_OVERFLOW, "level exceeds 2^31 - 1 boxes");
  IA_HIP(c, hipSetDevice(c->device));
  reset_bump(c);
  HitRec* recs = bump<HitRec>(c, size_t(std::max(1, n_hits)));
  if (!recs) return fail(c, IA_ERR_NOMEM, "scratch too small for %d hits", n_hits);
  hipStream_t s = as_stream(stream);
  Persistent* ps = persistent(c);
  if (n_hits > 0)
    hipLaunchKernelGGL(ia::k_prep, dim3((n_hits + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<const double*>(d_hits), d_active, n_hits, recs, nullptr, 0, &ps->status,
                       &ps->n_bad, nullptr, nullptr, nullptr, BoxD{}, nullptr);
  // the pre-pass flags, when the remaining scratch holds them (results do not depend on it)
  const size_t flag_cap = size_t(sh.n_parents) * sh.m012 * size_t(std::max(0, n_hits));
  uint8_t* flags = (n_hits > 0 && use_filter(c, sh)) ? bump<uint8_t>(c, flag_cap) : nullptr;
  const BoxD* par = reinterpret_cast<const BoxD*>(d_parents);
  const uint8_t* fl = launch_filter(c, recs, n_hits, par, sh, flags, flags ? flag_cap : 0, nullptr, s);
  return launch_vote(c, recs, n_hits, par, sh, d_votes, nullptr, 0, nullptr, fl, nullptr, s);
}

ia_status ia_refine(ia_ctx* c, const ia_box* d_parents, int32_t n_parents, const int32_t split[5],
                    const uint16_t* d_votes, int32_t vote_bound, int32_t top_k, ia_box* d_selected,
                    int64_t* d_selected_index, uint16_t* d_selected_votes, void* stream) {
  if (!c) return IA_ERR_INVALID;
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
  return launch_estimate(c, par, sh, d_votes, first, first_v, part, reinterpret_cast<ia::EstimateOut*>(d_out),
                         nullptr, nullptr, 0, 0.0, nullptr, nullptr, 0, nullptr, s);
}

ia_status ia_find_helices(ia_ctx* c, const ia_hit* d_hits, const int32_t* h_off, int32_t n_events,
                          const ia_schedule* sc, ia_helix* d_out, int32_t max_per_event, int32_t* d_n_out,
                          int32_t* d_assigned, void* stream) {
  if (!c) return IA_ERR_INVALID;
  if (!h_off || !sc || !d_out || !d_n_out) return fail(c, IA_ERR_INVALID, "null pointer argument");
  if (n_events < 0) return fail(c, IA_ERR_INVALID, "n_events %d < 0", n_events);
  if (max_per_event < 1) return fail(c, IA_ERR_INVALID, "max_per_event %d < 1", max_per_event);
  if (sc->n_refine < 0 || sc->n_refine >= IA_MAX_LEVELS) return fail(c, IA_ERR_INVALID, "n_refine %d", sc->n_refine);
  if (sc->top_k < 1 || sc->top_k > kMaxTopK) return fail(c, IA_ERR_INVALID, "top_k %d", sc->top_k);
  if (sc->n_helix_max < 0) return fail(c, IA_ERR_INVALID, "n_helix_max %d", sc->n_helix_max);
  if (!(sc->hitfind_scale >= 0.0)) return fail(c, IA_ERR_INVALID, "hitfind_scale");
  for (int j = 0; j < 5; ++j)
    if (!(sc->range.lo[j] <= sc->range.hi[j])) return fail(c, IA_ERR_INVALID, "range dimension %d: lo > hi", j);
  for (int l = 0; l <= sc->n_refine; ++l)
    if (sc->prec[l] != IA_FP64) return fail(c, IA_ERR_UNSUPPORTED, "precision %d at level %d", sc->prec[l], l);
  int32_t max_hits = 0;
  for (int32_t e = 0; e < n_events; ++e) {
    const int32_t n = h_off[e + 1] - h_off[e];
    if (n < 0 || n > kMaxHits) return fail(c, IA_ERR_INVALID, "event %d has %d hits", e, n);
    max_hits = std::max(max_hits, n);
  }
  if (max_hits > 0 && !d_hits) return fail(c, IA_ERR_INVALID, "d_hits is NULL");
  Shape sh0, shr;
  if (!make_shape(sc->bins, 1, &sh0)) return fail(c, IA_ERR_OVERFLOW, "level-0 grid exceeds 2^31 - 1 boxes");
  if (!make_shape(sc->split, sc->top_k, &shr)) return fail(c, IA_ERR_OVERFLOW, "refinement level too large");
  if (sh0.n_boxes > kMaxEstimateBoxes || shr.n_boxes > kMaxEstimateBoxes)
    return fail(c, IA_ERR_OVERFLOW, "a level exceeds %lld boxes", static_cast<long long>(kMaxEstimateBoxes));
  IA_HIP(c, hipSetDevice(c->device));
  const int32_t K = sc->top_k;
  const int64_t nt0 = int64_t(sh0.n_parents) * sh0.m012, ntr = int64_t(shr.n_parents) * shr.m012;
  FindLayout L;
  layout_find(std::max<int64_t>(sh0.n_boxes, shr.n_boxes), std::max(nt0, ntr), K, max_hits, &L);
  if (L.total > c->arena_bytes)
    return fail(c, IA_ERR_NOMEM, "scratch too small: need %zu bytes, have %zu", L.total, c->arena_bytes);
  char* a = c->arena;
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
  int32_t* wg_max = reinterpret_cast<int32_t*>(a + L.wg_max);
  hipStream_t s = as_stream(stream);
  Persistent* ps = persistent(c);
  BoxD rb;
  std::memcpy(&rb, &sc->range, sizeof rb);
  for (int32_t e = 0; e < n_events; ++e) {
    const int32_t n = h_off[e + 1] - h_off[e];
    const int32_t n_bins = n + 1;
    const double* hits = reinterpret_cast<const double*>(d_hits) + 8 * int64_t(h_off[e]);
    int32_t* assigned = d_assigned ? d_assigned + h_off[e] : nullptr;
    ia::HelixOut* out = reinterpret_cast<ia::HelixOut*>(d_out) + int64_t(e) * max_per_event;
    int32_t* n_out = d_n_out + e;
    const int32_t pg = std::max(1, (std::max(n, n_bins) + 255) / 256);
    hipLaunchKernelGGL(ia::k_prep, dim3(pg), dim3(256), 0, s, hits, nullptr, n, recs, hist, n_bins, &ps->status,
                       &ps->n_bad, ev, n_out, range, rb, assigned);
    for (int32_t pass = 0; pass < std::min(sc->n_helix_max, max_per_event); ++pass) {
      const BoxD* par = range;
      Shape sh = sh0;
      BoxD* sel = selA;
      for (int32_t lev = 0; lev <= sc->n_refine; ++lev) {
        const uint8_t* fl = launch_filter(c, recs, n, par, sh, flags, L.flag_cap, ev, s);
        int32_t bx = 0;
        ia_status st = launch_vote(c, recs, n, par, sh, votes, hist, n_bins, ev, fl, wg_max, s, &bx);
        if (st != IA_OK) return st;
        const uint32_t n_wg = (sh.n_boxes + bx - 1) / bx;
        hipLaunchKernelGGL(ia::k_select_wg, dim3(1), dim3(ia::kWG), 0, s, votes, sh.n_boxes, hist, n_bins, K, wg_max,
                           n_wg, bx, par, sh, sel, sel_idx, sel_v, ev, lev == 0 ? std::max(sc->v_min, 0) : 0);
        IA_HIP(c, hipGetLastError());
        if (lev == sc->n_refine) break;
        const int32_t k_eff = static_cast<int32_t>(std::min<int64_t>(K, sh.n_boxes));
        if (!make_shape(sc->split, k_eff, &sh)) return fail(c, IA_ERR_OVERFLOW, "split too large");
        par = sel;
        sel = (sel == selA) ? selB : selA;
      }
      ia_status st = launch_estimate(c, par, sh, votes, sel, sel_v, part, nullptr, ev, recs, n, sc->hitfind_scale,
                                     assigned, out, max_per_event, n_out, s);
      if (st != IA_OK) return st;
    }
  }
  return IA_OK;
}

}  // extern "C"
