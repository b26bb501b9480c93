"""Loader of the host-side check harness (the HIP library's vote arithmetic
compiled for the CPU).  Test infrastructure only."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ia_hostcheck.hip")
LIB = os.path.join(HERE, "libia_hostcheck.so")
ROOT = os.path.dirname(os.path.dirname(HERE))
DEPS = [SRC] + [os.path.join(ROOT, "paper_2401_04576_amd", "csrc", f) for f in ("ia_math.hpp", "ia_kernels.hpp")]
FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
         "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(force=True):
    stale = not os.path.exists(LIB) or any(os.path.getmtime(d) > os.path.getmtime(LIB) for d in DEPS)
    if force or stale:
        tmp = LIB + ".tmp"
        subprocess.check_call([os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), *FLAGS, "-o", tmp, SRC],
                              stderr=subprocess.DEVNULL)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.hc_vote_level.restype = C.c_int32
        L.hc_vote_level.argtypes = [P, C.c_int32, P, C.c_int32, P, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                    C.c_int32, C.c_int32, P, P]
        L.hc_g_pairs.restype = C.c_int32
        L.hc_g_pairs.argtypes = [P, C.c_int32, P, P, P]
        L.hc_encl_pairs.restype = C.c_int32
        L.hc_encl_pairs.argtypes = [P, C.c_int32, P, P, P]
        L.hc_e_magnitude.restype = C.c_int32
        L.hc_e_magnitude.argtypes = [P, P, P, C.c_uint32, P]
        _lib = L
    return _lib


def e_magnitude(hit, parent, split, tc):
    """(status, M, eps bound, discriminant bound) of the magnitude bound of
    d^Ax for one stereo hit over triple tc of `parent` split by `split`."""
    h = np.ascontiguousarray(np.atleast_1d(hit)).view(np.float64).reshape(-1, 8)[0].copy()
    p = np.atleast_1d(parent)
    pa = np.ascontiguousarray(np.concatenate([p["lo"], p["hi"]], axis=1)[0], dtype=np.float64)
    sp = np.ascontiguousarray(split, dtype=np.int32)
    out = np.zeros(3)
    rc = lib().hc_e_magnitude(h.ctypes.data, pa.ctypes.data, sp.ctypes.data, int(tc), out.ctypes.data)
    return int(rc), float(out[0]), float(out[1]), float(out[2])


def vote_level(hits, parents, split, filter_on, f32=False, slack=1e-6, prune_k=0, parent_filter=False, ties=False):
    h = np.ascontiguousarray(hits).view(np.float64).reshape(-1, 8).copy() if len(hits) else np.zeros((0, 8))
    p = np.atleast_1d(parents)
    pa = np.ascontiguousarray(np.concatenate([p["lo"], p["hi"]], axis=1), dtype=np.float64)
    sp = np.ascontiguousarray(split, dtype=np.int32)
    nb = pa.shape[0] * int(np.prod(sp.astype(np.int64)))
    votes = np.zeros(nb, dtype=np.uint16)
    stats = np.zeros(10, dtype=np.int64)
    rc = lib().hc_vote_level(h.ctypes.data, h.shape[0], pa.ctypes.data, pa.shape[0], sp.ctypes.data,
                             1 if filter_on else 0, 1 if f32 else 0, float(slack), int(prune_k),
                             1 if ties else 0, 1 if parent_filter else 0, votes.ctypes.data, stats.ctypes.data)
    assert rc == 0
    return votes, stats


def g_pairs(hits, parent, split):
    """(G, outer G) intervals of every (triple, hit) pair of one parent's
    level, shape (triples, hits, 4): G.lo, G.hi, Go.lo, Go.hi."""
    h = np.ascontiguousarray(hits).view(np.float64).reshape(-1, 8).copy()
    p = np.atleast_1d(parent)
    pa = np.ascontiguousarray(np.concatenate([p["lo"], p["hi"]], axis=1)[0], dtype=np.float64)
    sp = np.ascontiguousarray(split, dtype=np.int32)
    n_tr = int(np.prod(sp[:3].astype(np.int64)))
    out = np.zeros((n_tr, h.shape[0], 4))
    assert lib().hc_g_pairs(h.ctypes.data, h.shape[0], pa.ctypes.data, sp.ctypes.data, out.ctypes.data) == 0
    return out


def encl_pairs(hits, parent, split):
    """FP64 and FP32 enclosures of d^Ax and the range of its values at the
    box centres, per (triple, hit, drift sign) of one parent's level: shape
    (triples, hits, 2, 10), rows as in hc_encl_pairs."""
    h = np.ascontiguousarray(hits).view(np.float64).reshape(-1, 8).copy()
    p = np.atleast_1d(parent)
    pa = np.ascontiguousarray(np.concatenate([p["lo"], p["hi"]], axis=1)[0], dtype=np.float64)
    sp = np.ascontiguousarray(split, dtype=np.int32)
    n_tr = int(np.prod(sp[:3].astype(np.int64)))
    out = np.zeros((n_tr, h.shape[0], 2, 10))
    assert lib().hc_encl_pairs(h.ctypes.data, h.shape[0], pa.ctypes.data, sp.ctypes.data, out.ctypes.data) == 0
    return out
