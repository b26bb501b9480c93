"""MI355X interval-arithmetic helix vote: Python binding of libia.

Thin ctypes marshalling over the C ABI of include/ia.h.  Every step of the
search runs in the HIP kernels of libia.so; PyTorch only provides device
memory and the stream.  Importing works without a GPU; calling anything
that needs libia raises IAError when the library is missing (there is no
fallback path).

Tensor layouts (all on the context's CUDA/HIP device):
  hits     float64 (N, 8)   x0 y0 z0 x1 y1 z1 drift band
  boxes    float64 (B, 10)  lo[5] then hi[5], order d0 phi0 kappa z0 tanl
  votes    uint16 (n_boxes,)
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["IAError", "Context", "Schedule", "vote_level", "refine", "estimate", "find_helices",
           "lib_path", "load", "FP64", "FP32", "HELIX_DTYPE", "ESTIMATE_DTYPE"]

HERE = os.path.dirname(os.path.abspath(__file__))
FP64, FP32, FP64X, IV = 0, 1, 2, 3   # FP64X: exact Phi of Eq. CSAXtoPHI_a; IV: sound whole-box d^Ax
MAX_LEVELS = 8

_STATUS = {0: "IA_OK", 1: "IA_ERR_INVALID", 2: "IA_ERR_NOMEM", 3: "IA_ERR_DEVICE",
           4: "IA_ERR_UNSUPPORTED", 5: "IA_ERR_OVERFLOW"}


class IAError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * 5), ("hi", C.c_double * 5)]


SCHED_TOPK, SCHED_WINDOW = 0, 1


class Schedule(C.Structure):
    _fields_ = [("range", Box), ("bins", C.c_int32 * 5), ("n_refine", C.c_int32), ("top_k", C.c_int32),
                ("split", C.c_int32 * 5), ("v_min", C.c_int32), ("n_helix_max", C.c_int32),
                ("hitfind_scale", C.c_double), ("prec", C.c_int32 * MAX_LEVELS),
                ("fp32_slack", C.c_double), ("mode", C.c_int32), ("forward", C.c_int32),
                ("move_level", C.c_int32), ("wdrop", C.c_int32), ("hitsel", C.c_int32),
                ("lbins", (C.c_int32 * 5) * MAX_LEVELS), ("disk", C.c_double)]

    @classmethod
    def make(cls, lo, hi, bins, n_refine=4, top_k=32, split=(4, 4, 4, 4, 4), v_min=10, n_helix_max=1,
             hitfind_scale=5.0, prec=None, fp32_slack=1e-6, mode=SCHED_TOPK, forward=False, move_level=-1,
             lbins=None, wdrop=0, hitsel=False, disk=0.0):
        """mode SCHED_WINDOW: level l >= 1 is the grid lbins[l] over a window built from all max-vote
        boxes of level l - 1; the reference point moves after move_level (see include/ia.h)."""
        s = cls()
        s.mode = int(mode)
        s.forward = int(bool(forward))
        s.move_level = int(move_level)
        s.wdrop = int(wdrop)
        s.hitsel = int(bool(hitsel))
        s.disk = float(disk)
        if lbins is not None:
            for l, b in enumerate(lbins):
                for j in range(5):
                    s.lbins[l][j] = int(b[j])
        for j in range(5):
            s.range.lo[j] = float(lo[j])
            s.range.hi[j] = float(hi[j])
            s.bins[j] = int(bins[j])
            s.split[j] = int(split[j])
        s.n_refine = int(n_refine)
        s.top_k = int(top_k)
        s.v_min = int(v_min)
        s.n_helix_max = int(n_helix_max)
        s.hitfind_scale = float(hitfind_scale)
        prec = [FP64] * MAX_LEVELS if prec is None else list(prec) + [FP64] * (MAX_LEVELS - len(prec))
        for l in range(MAX_LEVELS):
            s.prec[l] = int(prec[l])
        s.fp32_slack = float(fp32_slack)
        return s


HELIX_DTYPE = np.dtype([("p", "f8", (5,)), ("err", "f8", (5,)), ("ref", "f8", (2,)), ("votes", "i4"),
                        ("n_assigned", "i4"), ("n_argmax", "i4"), ("status", "i4")])
ESTIMATE_DTYPE = np.dtype([("p", "f8", (5,)), ("err", "f8", (5,)), ("vmax", "i4"), ("n_argmax", "i4")])

_lib = None


def lib_path():
    return os.path.join(HERE, "libia.so")


def load():
    """Load libia.so; raise IAError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise IAError(4, f"{path} is missing: build it with __graft_entry__.build() "
                         "or python -m paper_2401_04576_amd.build")
    L = C.CDLL(path)
    P, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    L.ia_ctx_create.restype = i32
    L.ia_ctx_create.argtypes = [C.POINTER(P), i32, sz]
    L.ia_ctx_destroy.restype = None
    L.ia_ctx_destroy.argtypes = [P]
    L.ia_last_error.restype = C.c_char_p
    L.ia_last_error.argtypes = [P]
    L.ia_ctx_status.restype = i32
    L.ia_ctx_status.argtypes = [P, C.POINTER(C.c_uint32), C.POINTER(i64)]
    L.ia_ctx_work.restype = i32
    L.ia_ctx_work.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.ia_ctx_set_work_counting.restype = i32
    L.ia_ctx_set_work_counting.argtypes = [P, i32]
    L.ia_ctx_classify_work.restype = i32
    L.ia_ctx_classify_work.argtypes = [P, C.POINTER(i64)]
    L.ia_ctx_profile_kernels.restype = i32
    L.ia_ctx_profile_kernels.argtypes = [P, C.POINTER(i64), C.POINTER(C.c_double)]
    L.ia_ctx_set_fp32_slack.restype = i32
    L.ia_ctx_set_fp32_slack.argtypes = [P, C.c_double]
    L.ia_ctx_set_vote_frame.restype = i32
    L.ia_ctx_set_vote_frame.argtypes = [P, i32, C.c_double, C.c_double, C.c_double]
    L.ia_ctx_clear_status.restype = i32
    L.ia_ctx_clear_status.argtypes = [P]
    L.ia_ctx_set_batch.restype = i32
    L.ia_ctx_set_batch.argtypes = [P, i32]
    L.ia_ctx_set_parent_filter.restype = i32
    L.ia_ctx_set_parent_filter.argtypes = [P, i32]
    L.ia_ctx_set_pruning.restype = i32
    L.ia_ctx_set_pruning.argtypes = [P, i32]
    L.ia_ctx_set_prefilter.restype = i32
    L.ia_ctx_set_prefilter.argtypes = [P, i32]
    L.ia_ctx_set_vote_tile.restype = i32
    L.ia_ctx_set_vote_tile.argtypes = [P, i32]
    L.ia_ctx_set_profiling.restype = i32
    L.ia_ctx_set_profiling.argtypes = [P, i32]
    L.ia_ctx_profile_read.restype = i32
    L.ia_ctx_profile_read.argtypes = [P, C.POINTER(i64), C.POINTER(C.c_double), C.POINTER(i64),
                                      C.POINTER(C.c_double)]
    L.ia_ctx_scratch_needed.restype = sz
    L.ia_ctx_scratch_needed.argtypes = [C.POINTER(Schedule), i32]
    L.ia_vote_level.restype = i32
    L.ia_vote_level.argtypes = [P, P, i32, P, P, i32, C.POINTER(i32), i32, P, P]
    L.ia_vote_level_noalloc.restype = i32
    L.ia_vote_level_noalloc.argtypes = [P, i32, P, P, i32, C.POINTER(i32), i32, P, P]
    L.ia_refine.restype = i32
    L.ia_refine.argtypes = [P, P, i32, C.POINTER(i32), P, i32, i32, P, P, P, P]
    L.ia_estimate.restype = i32
    L.ia_estimate.argtypes = [P, P, i32, C.POINTER(i32), P, P, P]
    L.ia_find_helices.restype = i32
    L.ia_find_helices.argtypes = [P, P, C.POINTER(i32), i32, C.POINTER(Schedule), P, i32, P, P, P]
    L.ia_ctx_autotune.restype = i32
    L.ia_ctx_autotune.argtypes = [P, P, C.POINTER(i32), i32, C.POINTER(Schedule), P, i32, P, P]
    L.ia_ctx_tuned.restype = i32
    L.ia_ctx_tuned.argtypes = [P, P, P, i32]
    L.ia_find_helices_dev.restype = i32
    L.ia_find_helices_dev.argtypes = [P, P, P, i32, i32, i64, C.POINTER(Schedule), P, i32, P, P, P]
    L.ia_pool_capacity.restype = i32
    L.ia_pool_capacity.argtypes = [P, i32, C.POINTER(Schedule), i32]
    L.ia_pool_create.restype = i32
    L.ia_pool_create.argtypes = [P, i32, i32, C.POINTER(Schedule), i32, P]
    L.ia_pool_destroy.restype = i32
    L.ia_pool_destroy.argtypes = [P]
    L.ia_pool_admit.restype = i32
    L.ia_pool_admit.argtypes = [P, i32, C.POINTER(i32), P, C.POINTER(i32), P]
    L.ia_pool_step.restype = i32
    L.ia_pool_step.argtypes = [P, P]
    L.ia_pool_poll.restype = i32
    L.ia_pool_poll.argtypes = [P, C.POINTER(i32), P]
    L.ia_pool_take.restype = i32
    L.ia_pool_take.argtypes = [P, i32, i32, P, i32, C.POINTER(i32), P]
    _lib = L
    return L


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _split(split):
    arr = (C.c_int32 * 5)(*[int(v) for v in split])
    return arr


def _check_dev(t, dtype, name, device):
    torch = _torch()
    if t.dtype != dtype:
        raise IAError(1, f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_cuda or t.device.index != device:
        raise IAError(1, f"{name}: must be on cuda:{device}")
    if not t.is_contiguous():
        raise IAError(1, f"{name}: must be contiguous")
    return t


class Context:
    """Owns the library context (device scratch) for one device and stream."""

    def __init__(self, device=0, scratch_bytes=64 << 20):
        L = load()
        self.device = int(device)
        h = C.c_void_p()
        st = L.ia_ctx_create(C.byref(h), self.device, int(scratch_bytes))
        if st != 0:
            raise IAError(st, "ia_ctx_create failed")
        self._h = h
        self._L = L

    def _check(self, st):
        if st != 0:
            raise IAError(st, self._L.ia_last_error(self._h).decode())

    def status(self):
        flags, nbad = C.c_uint32(), C.c_int64()
        self._check(self._L.ia_ctx_status(self._h, C.byref(flags), C.byref(nbad)))
        return int(flags.value), int(nbad.value)

    def work(self):
        """(stereo box evaluations, staged pairs) at FP64 levels, then the same
        two at FP32 levels, since the last clear_status()."""
        a, b, f, g = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self._L.ia_ctx_work(self._h, C.byref(a), C.byref(b), C.byref(f), C.byref(g)))
        return int(a.value), int(b.value), int(f.value), int(g.value)

    def set_work_counting(self, enable=True):
        """Classification launches count their work (a slower variant) while enabled."""
        self._check(self._L.ia_ctx_set_work_counting(self._h, 1 if enable else 0))

    def classify_work(self):
        """Classification work counted (set_work_counting) since the last clear_status(): {"fp64": {...},
        "fp32": {...}} with counts of outer residuals G, axial tests, exact G,
        stereo pair magnitudes and magnitude bounds (first stage), and
        deferred pairs, d^Ax enclosures and inclusion proofs (second stage)."""
        a = (C.c_int64 * 16)()
        self._check(self._L.ia_ctx_classify_work(self._h, a))
        keys = ("G", "axial", "G_exact", "pairq", "magnitudes", "deferred", "enclosures", "inclusions")
        return {p: {k: int(a[8 * i + j]) for j, k in enumerate(keys)} for i, p in enumerate(("fp64", "fp32"))}

    def set_fp32_slack(self, slack=1e-6):
        """Band widening of vote_level at FP32 (m)."""
        self._check(self._L.ia_ctx_set_fp32_slack(self._h, float(slack)))

    def set_vote_frame(self, forward=False, ref=(0.0, 0.0), disk=0.0):
        """forward-hit test, reference point and disk condition of vote_level"""
        self._check(self._L.ia_ctx_set_vote_frame(self._h, int(forward), float(ref[0]), float(ref[1]),
                                                  float(disk)))

    def clear_status(self):
        self._check(self._L.ia_ctx_clear_status(self._h))

    def set_vote_tile(self, boxes_per_workgroup=0):
        """Force the vote kernel's boxes per workgroup (256, 128, 64) or 0 for automatic."""
        self._check(self._L.ia_ctx_set_vote_tile(self._h, int(boxes_per_workgroup)))

    def set_batch(self, max_events=65535):
        """Maximum events per batched launch of find_helices."""
        self._check(self._L.ia_ctx_set_batch(self._h, int(max_events)))

    def set_pruning(self, enable=True, probe=True):
        """find_helices: skip triples whose vote upper bound cannot reach the
        selection; with `probe` (window schedule) the threshold is raised by
        the largest vote among the triples with the largest upper bounds,
        voted first."""
        self._check(self._L.ia_ctx_set_pruning(self._h, (2 if probe else 1) if enable else 0))

    def autotune(self, hits, offsets, sched, max_per_event=16, stream=None):
        """Pick the vote tile per level size by timing a sample batch; returns {level boxes: tile}."""
        torch = _torch()
        _check_dev(hits, torch.float64, "hits", self.device)
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
        n_events = off.shape[0] - 1
        out = torch.zeros(max(1, n_events * max_per_event) * HELIX_DTYPE.itemsize, dtype=torch.uint8,
                          device=hits.device)
        n_out = torch.zeros(max(1, n_events), dtype=torch.int32, device=hits.device)
        self._check(self._L.ia_ctx_autotune(self._h, _ptr(hits), off.ctypes.data_as(C.POINTER(C.c_int32)),
                                            int(n_events), C.byref(sched), _ptr(out), int(max_per_event),
                                            _ptr(n_out), _stream_handle(stream)))
        nb = np.zeros(64, dtype=np.uint32)
        tl = np.zeros(64, dtype=np.int32)
        n = self._L.ia_ctx_tuned(self._h, nb.ctypes.data, tl.ctypes.data, 64)
        return {int(nb[i]): int(tl[i]) for i in range(min(n, 64))}

    def set_parent_filter(self, enable=True):
        """find_helices: parent-level exclusion of hits at refinement levels."""
        self._check(self._L.ia_ctx_set_parent_filter(self._h, 1 if enable else 0))

    def set_prefilter(self, mode=-1):
        """(triple, hit) classification proofs: -1 or 1 on, 0 off."""
        self._check(self._L.ia_ctx_set_prefilter(self._h, int(mode)))

    def set_profiling(self, enable=True):
        self._check(self._L.ia_ctx_set_profiling(self._h, 1 if enable else 0))

    def profile_read(self):
        """(FP64 vote launches, their ms, FP32 vote launches, their ms) since the last read."""
        n, ms, n32, ms32 = C.c_int64(), C.c_double(), C.c_int64(), C.c_double()
        self._check(self._L.ia_ctx_profile_read(self._h, C.byref(n), C.byref(ms), C.byref(n32), C.byref(ms32)))
        return int(n.value), float(ms.value), int(n32.value), float(ms32.value)

    def profile_kernels(self):
        """{(kernel, prec): (launches, ms)} for kernel in ("vote", "classify",
        "classify_defer") and prec in ("fp64", "fp32"), since the last read
        (clears the record)."""
        n = (C.c_int64 * 6)()
        ms = (C.c_double * 6)()
        self._check(self._L.ia_ctx_profile_kernels(self._h, n, ms))
        return {(k, p): (int(n[2 * i + j]), float(ms[2 * i + j]))
                for i, k in enumerate(("vote", "classify", "classify_defer")) for j, p in enumerate(("fp64", "fp32"))}

    def close(self):
        if getattr(self, "_h", None):
            self._L.ia_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def scratch_needed(sched, max_hits):
        return int(load().ia_ctx_scratch_needed(C.byref(sched), int(max_hits)))


def vote_level(ctx, hits, parents, split, votes=None, active=None, prec=FP64, stream=None):
    """Votes of `hits` for every child box of `parents` split by `split`."""
    torch = _torch()
    _check_dev(hits, torch.float64, "hits", ctx.device)
    _check_dev(parents, torch.float64, "parents", ctx.device)
    nb = parents.shape[0] * int(np.prod([int(s) for s in split]))
    if votes is None:
        votes = torch.empty(nb, dtype=torch.uint16, device=hits.device)
    _check_dev(votes, torch.uint16, "votes", ctx.device)
    if votes.numel() < nb:
        raise IAError(1, "votes too small")
    if active is not None:
        _check_dev(active, torch.uint8, "active", ctx.device)
    ctx._check(ctx._L.ia_vote_level(ctx._h, _ptr(hits), int(hits.shape[0]), _ptr(active), _ptr(parents),
                                    int(parents.shape[0]), _split(split), int(prec), _ptr(votes),
                                    _stream_handle(stream)))
    return votes


NOALLOC_SCRATCH_BYTES = 64 << 20


def vote_level_noalloc(hits, parents, split, votes, active=None, prec=FP64, stream=None):
    """vote_level without a context: the library's scratch is a fixed device
    array and the call allocates nothing (`votes` is the caller's).  Calls
    that overlap on one GPU race."""
    torch = _torch()
    dev = hits.device.index or 0
    _check_dev(hits, torch.float64, "hits", dev)
    _check_dev(parents, torch.float64, "parents", dev)
    _check_dev(votes, torch.uint16, "votes", dev)
    nb = parents.shape[0] * int(np.prod([int(s) for s in split]))
    if votes.numel() < nb:
        raise IAError(1, "votes too small")
    if active is not None:
        _check_dev(active, torch.uint8, "active", dev)
    L = load()
    with torch.cuda.device(dev):   # the library uses the current device's array
        st = L.ia_vote_level_noalloc(_ptr(hits), int(hits.shape[0]), _ptr(active), _ptr(parents),
                                     int(parents.shape[0]), _split(split), int(prec), _ptr(votes),
                                     _stream_handle(stream))
    if st != 0:
        raise IAError(st, L.ia_last_error(None).decode())
    return votes


def refine(ctx, parents, split, votes, vote_bound, top_k, stream=None):
    """Top-k boxes by (votes desc, index asc): (boxes (k, 10), index (k,), votes (k,))."""
    torch = _torch()
    _check_dev(parents, torch.float64, "parents", ctx.device)
    _check_dev(votes, torch.uint16, "votes", ctx.device)
    nb = parents.shape[0] * int(np.prod([int(s) for s in split]))
    k = min(int(top_k), nb)
    dev = votes.device
    sel = torch.empty((k, 10), dtype=torch.float64, device=dev)
    idx = torch.empty(k, dtype=torch.int64, device=dev)
    sv = torch.empty(k, dtype=torch.uint16, device=dev)
    ctx._check(ctx._L.ia_refine(ctx._h, _ptr(parents), int(parents.shape[0]), _split(split), _ptr(votes),
                                int(vote_bound), int(top_k), _ptr(sel), _ptr(idx), _ptr(sv),
                                _stream_handle(stream)))
    return sel, idx, sv


def estimate(ctx, parents, split, votes, stream=None):
    """Estimate from the max-vote boxes; returns a uint8 device tensor holding one ESTIMATE_DTYPE record."""
    torch = _torch()
    _check_dev(parents, torch.float64, "parents", ctx.device)
    _check_dev(votes, torch.uint16, "votes", ctx.device)
    out = torch.zeros(ESTIMATE_DTYPE.itemsize, dtype=torch.uint8, device=votes.device)
    ctx._check(ctx._L.ia_estimate(ctx._h, _ptr(parents), int(parents.shape[0]), _split(split), _ptr(votes),
                                  _ptr(out), _stream_handle(stream)))
    return out


def decode(raw, dtype):
    """Device bytes -> numpy structured array (synchronises)."""
    return np.frombuffer(raw.cpu().numpy().tobytes(), dtype=dtype)


def find_helices(ctx, hits, offsets, sched, max_per_event=16, want_assigned=True, stream=None,
                 out=None, n_out=None, assigned=None):
    """Run the whole search on the events of `hits` (CSR `offsets`, host ints).

    Returns device tensors (helices as raw bytes, n_out int32, assigned int32 or None).
    Output tensors may be passed in to avoid allocations."""
    torch = _torch()
    _check_dev(hits, torch.float64, "hits", ctx.device)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
    n_events = off.shape[0] - 1
    # the C ABI takes no hit count: the offsets must stay inside `hits`
    if n_events < 0 or (n_events > 0 and (off[0] < 0 or off[-1] > hits.shape[0] or np.any(np.diff(off) < 0))):
        raise IAError(1, "offsets must be non-decreasing within [0, hits.shape[0]]")
    dev = hits.device
    if out is None:
        out = torch.zeros(max(1, n_events * max_per_event) * HELIX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    if n_out is None:
        n_out = torch.zeros(max(1, n_events), dtype=torch.int32, device=dev)
    if assigned is None and want_assigned:
        assigned = torch.full((max(1, hits.shape[0]),), -1, dtype=torch.int32, device=dev)
    if out.numel() < n_events * max_per_event * HELIX_DTYPE.itemsize or n_out.numel() < n_events:
        raise IAError(1, "output tensors too small")
    if assigned is not None and assigned.numel() < hits.shape[0]:
        raise IAError(1, "assigned too small")
    ctx._check(ctx._L.ia_find_helices(ctx._h, _ptr(hits), off.ctypes.data_as(C.POINTER(C.c_int32)), int(n_events),
                                      C.byref(sched), _ptr(out), int(max_per_event), _ptr(n_out), _ptr(assigned),
                                      _stream_handle(stream)))
    return out, n_out, assigned


def find_helices_dev(ctx, hits, d_off, max_hits, sched, out, n_out, assigned=None, max_per_event=16, stream=None):
    """The search with device offsets (int32 tensor of n_events + 1), enqueuing
    kernels only, so it can be captured in a HIP graph (torch.cuda.graph) and
    replayed on new contents of the same buffers."""
    torch = _torch()
    _check_dev(hits, torch.float64, "hits", ctx.device)
    _check_dev(d_off, torch.int32, "d_off", ctx.device)
    n_events = d_off.numel() - 1
    if out.numel() < n_events * max_per_event * HELIX_DTYPE.itemsize or n_out.numel() < n_events:
        raise IAError(1, "output tensors too small")
    if assigned is not None and assigned.numel() < hits.shape[0]:
        raise IAError(1, "assigned too small")
    ctx._check(ctx._L.ia_find_helices_dev(ctx._h, _ptr(hits), _ptr(d_off), int(n_events), int(max_hits),
                                          int(hits.shape[0]), C.byref(sched), _ptr(out), int(max_per_event),
                                          _ptr(n_out), _ptr(assigned), _stream_handle(stream)))
    return out, n_out, assigned


class Pool:
    """A resident pool of `rows` event rows of up to `max_hits` hits on a
    context (ia_pool_*): events are admitted into free rows at any time and
    every step() runs one helix pass over all rows still searching."""

    def __init__(self, ctx, rows, max_hits, sched, max_per_event=10, stream=None):
        self.ctx, self.rows, self.max_hits = ctx, int(rows), int(max_hits)
        self.max_out = min(int(sched.n_helix_max), int(max_per_event))
        self.stream = stream
        ctx._check(ctx._L.ia_pool_create(ctx._h, self.rows, self.max_hits, C.byref(sched), int(max_per_event),
                                         _stream_handle(stream)))
        self._state = np.zeros(2 * self.rows, dtype=np.int32)

    @staticmethod
    def capacity(ctx, max_hits, sched, max_per_event=10):
        """Rows of max_hits hits that fit the context's arena."""
        return int(ctx._L.ia_pool_capacity(ctx._h, int(max_hits), C.byref(sched), int(max_per_event)))

    def admit(self, rows, hits, offsets):
        """Events j = hits[offsets[j]:offsets[j+1]] (device float64 (n, 8)
        tensor, host offsets) into rows[j]."""
        torch = _torch()
        _check_dev(hits, torch.float64, "hits", self.ctx.device)
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
        if off.shape[0] != r.shape[0] + 1 or (r.shape[0] and (off[0] < 0 or off[-1] > hits.shape[0]
                                                              or np.any(np.diff(off) < 0))):
            raise IAError(1, "offsets must be len(rows) + 1 non-decreasing values within the hits")
        self.ctx._check(self.ctx._L.ia_pool_admit(self.ctx._h, int(r.shape[0]), r.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  _ptr(hits), off.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  _stream_handle(self.stream)))

    def step(self):
        self.ctx._check(self.ctx._L.ia_pool_step(self.ctx._h, _stream_handle(self.stream)))

    def poll(self):
        """(done flags, helices written) per row; synchronises the stream."""
        self.ctx._check(self.ctx._L.ia_pool_poll(self.ctx._h, self._state.ctypes.data_as(C.POINTER(C.c_int32)),
                                                 _stream_handle(self.stream)))
        return self._state[0::2].copy(), self._state[1::2].copy()

    def take(self, row, n_helices, n_hits):
        """(helices, assigned) of a finished row."""
        out = np.zeros(max(1, n_helices), dtype=HELIX_DTYPE)
        ass = np.zeros(max(1, n_hits), dtype=np.int32)
        self.ctx._check(self.ctx._L.ia_pool_take(self.ctx._h, int(row), int(n_helices), out.ctypes.data_as(C.c_void_p),
                                                 int(n_hits), ass.ctypes.data_as(C.POINTER(C.c_int32)),
                                                 _stream_handle(self.stream)))
        return out[:n_helices], ass[:n_hits]

    def close(self):
        if self.ctx is not None and self.ctx._h:
            self.ctx._L.ia_pool_destroy(self.ctx._h)
        self.ctx = None

