"""ctypes binding of the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does.
The C source (ia_oracle.c) follows the paper's equations directly and
shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ia_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

HIT_DTYPE = np.dtype([("x0", "f8"), ("y0", "f8"), ("z0", "f8"),
                      ("x1", "f8"), ("y1", "f8"), ("z1", "f8"),
                      ("drift", "f8"), ("band", "f8")])
BOX_DTYPE = np.dtype([("lo", "f8", (5,)), ("hi", "f8", (5,))])
PREP_DTYPE = np.dtype([("valid", "i4"), ("axial", "i4"), ("px", "f8"), ("py", "f8"),
                       ("tant", "f8"), ("sphis", "f8"), ("cphis", "f8"), ("r", "f8"),
                       ("phip", "f8"), ("r2lo", "f8"), ("r2hi", "f8"), ("d", "f8"),
                       ("band", "f8")])
SCHED_DTYPE = np.dtype([("range", BOX_DTYPE), ("bins", "i4", (5,)), ("n_refine", "i4"),
                        ("top_k", "i4"), ("split", "i4", (5,)), ("v_min", "i4"),
                        ("n_helix_max", "i4"), ("hitfind_scale", "f8"), ("prec", "i4", (8,)),
                        ("fp32_slack", "f8"), ("mode", "i4"), ("forward", "i4"),
                        ("move_level", "i4"), ("wdrop", "i4"), ("hitsel", "i4"),
                        ("lbins", "i4", (8, 5)), ("disk", "f8")], align=True)
FP64, FP32, FP64X, IV = 0, 1, 2, 3   # FP64X: exact Phi of Eq. CSAXtoPHI_a; IV: sound whole-box d^Ax
TOPK, WINDOW = 0, 1
HELIX_DTYPE = np.dtype([("p", "f8", (5,)), ("err", "f8", (5,)), ("ref", "f8", (2,)), ("votes", "i4"),
                        ("n_assigned", "i4"), ("n_argmax", "i4"), ("pad", "i4")])
MAX_LEVELS, MAX_K, MAX_PASSES = 8, 64, 16
TRACE_DTYPE = np.dtype([("n_passes", "i4"),
                        ("vmax", "i4", (MAX_PASSES, MAX_LEVELS)),
                        ("n_argmax", "i4", (MAX_PASSES, MAX_LEVELS)),
                        ("selected", BOX_DTYPE, (MAX_PASSES, MAX_LEVELS, MAX_K)),
                        ("selected_index", "i8", (MAX_PASSES, MAX_LEVELS, MAX_K)),
                        ("grid", BOX_DTYPE, (MAX_PASSES, MAX_LEVELS)),
                        ("ref", "f8", (MAX_PASSES, MAX_LEVELS, 2))], align=True)

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-fopenmp", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (scalar, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None
_P = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        L.or_sin.restype = d; L.or_sin.argtypes = [d]
        L.or_cos.restype = d; L.or_cos.argtypes = [d]
        L.or_atan2.restype = d; L.or_atan2.argtypes = [d, d]
        L.or_wdn.restype = d; L.or_wdn.argtypes = [d]
        L.or_wup.restype = d; L.or_wup.argtypes = [d]
        L.or_sin_encl.restype = None; L.or_sin_encl.argtypes = [d, d, _P, _P]
        L.or_imul.restype = None; L.or_imul.argtypes = [d, d, d, d, _P, _P]
        L.or_isqr.restype = None; L.or_isqr.argtypes = [d, d, _P, _P]
        L.or_prep_hit.restype = i32; L.or_prep_hit.argtypes = [_P, _P]
        L.or_box_child.restype = None; L.or_box_child.argtypes = [_P, _P, i64, _P]
        L.or_stereo_e.restype = i32; L.or_stereo_e.argtypes = [_P, _P, i32, _P, _P]
        L.or_stereo_e_x.restype = i32; L.or_stereo_e_x.argtypes = [_P, _P, i32, i32, _P, _P]
        L.or_pair_vote.restype = i32; L.or_pair_vote.argtypes = [_P, _P, _P]
        L.or_pair_vote_x.restype = i32; L.or_pair_vote_x.argtypes = [_P, _P, i32, _P]
        L.or_stereo_encl.restype = i32; L.or_stereo_encl.argtypes = [_P, _P, i32, _P, _P]
        L.or_pair_vote_iv.restype = i32; L.or_pair_vote_iv.argtypes = [_P, _P]
        L.or_vote_level.restype = None
        L.or_vote_level.argtypes = [_P, i32, _P, _P, i32, _P, _P, i32]
        L.or_vote_level_prec.restype = None
        L.or_vote_level_prec.argtypes = [_P, i32, _P, _P, i32, _P, i32, d, _P, i32]
        f = C.c_float
        L.or_rd32.restype = f; L.or_rd32.argtypes = [d]
        L.or_ru32.restype = f; L.or_ru32.argtypes = [d]
        L.or_wdn32.restype = f; L.or_wdn32.argtypes = [f]
        L.or_wup32.restype = f; L.or_wup32.argtypes = [f]
        L.or_sinf1.restype = f; L.or_sinf1.argtypes = [f]
        L.or_sinf.restype = f; L.or_sinf.argtypes = [f]
        L.or_cosf.restype = f; L.or_cosf.argtypes = [f]
        L.or_atan2f.restype = f; L.or_atan2f.argtypes = [f, f]
        L.or_sin_encl32.restype = None; L.or_sin_encl32.argtypes = [f, f, _P, _P]
        L.or_pair_G32.restype = None; L.or_pair_G32.argtypes = [_P, _P, _P, _P]
        L.or_cosf1.restype = f; L.or_cosf1.argtypes = [f]
        L.or_stereo_e32.restype = i32; L.or_stereo_e32.argtypes = [_P, _P, i32, _P, _P]
        L.or_pair_vote32.restype = i32; L.or_pair_vote32.argtypes = [_P, _P, d, _P]
        L.or_topk.restype = i32; L.or_topk.argtypes = [_P, i64, i32, _P, _P]
        L.or_estimate.restype = i32
        L.or_estimate.argtypes = [_P, i32, _P, _P, C.c_uint16, _P, _P]
        L.or_prep_hit_ref.restype = i32; L.or_prep_hit_ref.argtypes = [_P, d, d, _P]
        L.or_forward.restype = i32; L.or_forward.argtypes = [_P, _P]
        L.or_frame_shift.restype = None; L.or_frame_shift.argtypes = [_P, d, d, _P]
        L.or_point_G.restype = d; L.or_point_G.argtypes = [_P, _P]
        L.or_vote_level_ex.restype = None
        L.or_vote_level_ex.argtypes = [_P, i32, _P, _P, i32, _P, i32, d, i32, d, d, d, _P, i32]
        L.or_disk.restype = i32; L.or_disk.argtypes = [_P, d, d, d]
        L.or_behind.restype = i32; L.or_behind.argtypes = [_P, d, d]
        L.or_estimate_ex.restype = i32
        L.or_estimate_ex.argtypes = [_P, i32, _P, _P, C.c_uint16, _P, _P, _P, _P]
        L.or_find_helices.restype = i32
        L.or_find_helices.argtypes = [_P, i32, _P, _P, i32, _P, _P, i32]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_P) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ----------------------------------------------------------------------------
# thin numpy wrappers
# ----------------------------------------------------------------------------
def sin(x):
    return lib().or_sin(float(x))


def cos(x):
    return lib().or_cos(float(x))


def atan2(y, x):
    return lib().or_atan2(float(y), float(x))


def wdn(x):
    return lib().or_wdn(float(x))


def wup(x):
    return lib().or_wup(float(x))


def sin_encl(a, b):
    lo, hi = C.c_double(), C.c_double()
    lib().or_sin_encl(float(a), float(b), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def imul(a, b):
    lo, hi = C.c_double(), C.c_double()
    lib().or_imul(float(a[0]), float(a[1]), float(b[0]), float(b[1]), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def isqr(a):
    lo, hi = C.c_double(), C.c_double()
    lib().or_isqr(float(a[0]), float(a[1]), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def prep_hits(hits, ref=(0.0, 0.0)):
    hits = _c(hits, HIT_DTYPE)
    out = np.zeros(hits.shape[0], dtype=PREP_DTYPE)
    for i in range(hits.shape[0]):
        lib().or_prep_hit_ref(_ptr(hits[i:i + 1]), float(ref[0]), float(ref[1]), _ptr(out[i:i + 1]))
    return out


def forward(prep, box):
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    box = _c(np.atleast_1d(box), BOX_DTYPE)
    return int(lib().or_forward(_ptr(prep), _ptr(box)))


def frame_shift(p, dx, dy):
    p = _c(p, np.float64)
    q = np.zeros(5)
    lib().or_frame_shift(_ptr(p), float(dx), float(dy), _ptr(q))
    return q


def point_G(prep, p):
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    return float(lib().or_point_G(_ptr(prep), _ptr(_c(p, np.float64))))


def make_box(lo, hi):
    b = np.zeros((), dtype=BOX_DTYPE)
    b["lo"] = lo
    b["hi"] = hi
    return b


def box_child(parent, split, child):
    parent = _c(np.atleast_1d(parent), BOX_DTYPE)
    split = _c(split, np.int32)
    out = np.zeros(1, dtype=BOX_DTYPE)
    lib().or_box_child(_ptr(parent), _ptr(split), int(child), _ptr(out))
    return out[0]


def stereo_e(prep, c, s, debug=False, exact=False):
    """d^Ax at the point c for drift sign s; exact: Phi from Eq. CSAXtoPHI_a."""
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    c = _c(c, np.float64)
    e = np.zeros(1)
    dbg = np.full(24, np.nan) if debug else None
    ok = lib().or_stereo_e_x(_ptr(prep), _ptr(c), int(s), 1 if exact else 0, _ptr(e), _ptr(dbg))
    if debug:
        return bool(ok), float(e[0]), dbg
    return bool(ok), float(e[0])


STEREO_DEBUG_NAMES = ["R", "xc", "yc", "Dx", "Dy", "RAx", "cAx", "sAx", "sinA", "cosA", "dphi",
                      "zA", "Phi1", "Phi2", "eps", "sinP", "cosP", "u", "delta", "sperp", "zS",
                      "ctau", "Q", "dhat"]


def pair_vote(prep, box, debug=False, exact=False):
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    box = _c(np.atleast_1d(box), BOX_DTYPE)
    dbg = np.full(8, np.nan) if debug else None
    v = lib().or_pair_vote_x(_ptr(prep), _ptr(box), 1 if exact else 0, _ptr(dbg))
    return (int(v), dbg) if debug else int(v)


def stereo_encl(prep, box, s):
    """(ok, lo, hi): enclosure of e = sgn(kappa) d^Ax over the whole box (IV levels)."""
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    box = _c(np.atleast_1d(box), BOX_DTYPE)
    lo, hi = np.zeros(1), np.zeros(1)
    ok = lib().or_stereo_encl(_ptr(prep), _ptr(box), int(s), _ptr(lo), _ptr(hi))
    return bool(ok), float(lo[0]), float(hi[0])


def pair_vote_iv(prep, box):
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    box = _c(np.atleast_1d(box), BOX_DTYPE)
    return int(lib().or_pair_vote_iv(_ptr(prep), _ptr(box)))


def disk(box, ref=(0.0, 0.0), radius=5e-3):
    box = _c(np.atleast_1d(box), BOX_DTYPE)
    return int(lib().or_disk(_ptr(box), float(ref[0]), float(ref[1]), float(radius)))


def behind(box, ref):
    box = _c(np.atleast_1d(box), BOX_DTYPE)
    return int(lib().or_behind(_ptr(box), float(ref[0]), float(ref[1])))


def vote_level(hits, parents, split, active=None, n_threads=0, prec=FP64, slack=1e-6, forward=False,
               ref=(0.0, 0.0), disk=0.0):
    hits = _c(hits, HIT_DTYPE)
    parents = _c(np.atleast_1d(parents), BOX_DTYPE)
    split = _c(split, np.int32)
    nb = parents.shape[0] * int(np.prod(split.astype(np.int64)))
    votes = np.zeros(nb, dtype=np.uint16)
    act = None if active is None else _c(active, np.uint8)
    lib().or_vote_level_ex(_ptr(hits), hits.shape[0], _ptr(act), _ptr(parents), parents.shape[0],
                           _ptr(split), int(prec), C.c_double(slack), int(forward),
                           float(ref[0]), float(ref[1]), float(disk), _ptr(votes), int(n_threads))
    return votes


def rd32(x):
    return np.float32(lib().or_rd32(C.c_double(x)))


def ru32(x):
    return np.float32(lib().or_ru32(C.c_double(x)))


def wdn32(x):
    return np.float32(lib().or_wdn32(C.c_float(x)))


def wup32(x):
    return np.float32(lib().or_wup32(C.c_float(x)))


def sinf1(x):
    return np.float32(lib().or_sinf1(C.c_float(x)))


def sinf(x):
    return np.float32(lib().or_sinf(C.c_float(x)))


def cosf(x):
    return np.float32(lib().or_cosf(C.c_float(x)))


def atan2f(y, x):
    return np.float32(lib().or_atan2f(C.c_float(y), C.c_float(x)))


def sin_encl32(a, b):
    lo, hi = np.zeros(1, dtype=np.float32), np.zeros(1, dtype=np.float32)
    lib().or_sin_encl32(C.c_float(a), C.c_float(b), _ptr(lo), _ptr(hi))
    return lo[0], hi[0]


def pair_G32(prep, box):
    """FP32 interval G of Eq. ApoVote over the box."""
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    box = _c(np.atleast_1d(box), BOX_DTYPE)
    lo, hi = np.zeros(1, dtype=np.float32), np.zeros(1, dtype=np.float32)
    lib().or_pair_G32(_ptr(prep), _ptr(box), _ptr(lo), _ptr(hi))
    return lo[0], hi[0]


def cosf1(x):
    return np.float32(lib().or_cosf1(C.c_float(x)))


def stereo_e32(prep, c, s, debug=False):
    """FP32-level d^Ax: (valid, e32) or (valid, e32, 24 float intermediates)."""
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    c = _c(c, np.float64)
    e = np.zeros(1, dtype=np.float32)
    dbg = np.full(24, np.nan, dtype=np.float32) if debug else None
    ok = lib().or_stereo_e32(_ptr(prep), _ptr(c), int(s), _ptr(e), _ptr(dbg))
    if debug:
        return bool(ok), e[0], dbg
    return bool(ok), e[0]


def pair_vote32(prep, box, slack=1e-6, debug=False):
    prep = _c(np.atleast_1d(prep), PREP_DTYPE)
    box = _c(np.atleast_1d(box), BOX_DTYPE)
    dbg = np.full(8, np.nan, dtype=np.float32) if debug else None
    v = lib().or_pair_vote32(_ptr(prep), _ptr(box), C.c_double(slack), _ptr(dbg))
    return (int(v), dbg) if debug else int(v)


def topk(votes, k):
    votes = _c(votes, np.uint16)
    idx = np.zeros(max(k, 1), dtype=np.int64)
    v = np.zeros(max(k, 1), dtype=np.uint16)
    kk = lib().or_topk(_ptr(votes), votes.shape[0], int(k), _ptr(idx), _ptr(v))
    return idx[:kk], v[:kk]


def estimate(parents, split, votes, vmax):
    parents = _c(np.atleast_1d(parents), BOX_DTYPE)
    split = _c(split, np.int32)
    votes = _c(votes, np.uint16)
    p = np.zeros(5)
    err = np.zeros(5)
    n = lib().or_estimate(_ptr(parents), parents.shape[0], _ptr(split), _ptr(votes),
                          int(vmax), _ptr(p), _ptr(err))
    return p, err, int(n)


def estimate_ex(parents, split, votes, vmax):
    """(p, err, n_argmax, union lo, union hi)"""
    parents = _c(np.atleast_1d(parents), BOX_DTYPE)
    split = _c(split, np.int32)
    votes = _c(votes, np.uint16)
    p, err, ulo, uhi = np.zeros(5), np.zeros(5), np.zeros(5), np.zeros(5)
    n = lib().or_estimate_ex(_ptr(parents), parents.shape[0], _ptr(split), _ptr(votes), int(vmax),
                             _ptr(p), _ptr(err), _ptr(ulo), _ptr(uhi))
    return p, err, int(n), ulo, uhi


def make_sched(lo, hi, bins, n_refine=4, top_k=32, split=(4, 4, 4, 4, 4), v_min=10,
               n_helix_max=1, hitfind_scale=5.0, prec=None, fp32_slack=1e-6, mode=TOPK, forward=False,
               move_level=-1, lbins=None, wdrop=0, hitsel=False, disk=0.0):
    """prec: per-level FP64 / FP32 / FP64X list (default all FP64).  mode WINDOW: level l >= 1 is
    a grid of lbins[l] over its window; the reference point moves after move_level."""
    s = np.zeros((), dtype=SCHED_DTYPE)
    s["mode"] = mode
    s["forward"] = int(bool(forward))
    s["move_level"] = move_level
    s["wdrop"] = wdrop
    s["hitsel"] = int(bool(hitsel))
    s["disk"] = disk
    if lbins is not None:
        for l, b in enumerate(lbins):
            s["lbins"][l] = b
    if prec is not None:
        s["prec"][:len(prec)] = prec
    s["fp32_slack"] = fp32_slack
    s["range"]["lo"] = lo
    s["range"]["hi"] = hi
    s["bins"] = bins
    s["n_refine"] = n_refine
    s["top_k"] = top_k
    s["split"] = split
    s["v_min"] = v_min
    s["n_helix_max"] = n_helix_max
    s["hitfind_scale"] = hitfind_scale
    return s


def find_helices(hits, sched, max_out=16, n_threads=0, want_trace=False):
    hits = _c(hits, HIT_DTYPE)
    sched = np.ascontiguousarray(np.atleast_1d(sched))
    out = np.zeros(max_out, dtype=HELIX_DTYPE)
    assigned = np.full(hits.shape[0], -1, dtype=np.int32)
    trace = np.zeros(1, dtype=TRACE_DTYPE) if want_trace else None
    n = lib().or_find_helices(_ptr(hits), hits.shape[0], _ptr(sched), _ptr(out), int(max_out),
                              _ptr(assigned), _ptr(trace), int(n_threads))
    res = (out[:n], assigned)
    return res + (trace[0],) if want_trace else res
