"""Host-side checks of the C ABI: the built library loads without a GPU and
exports every function include/ia.h declares; host-checkable argument errors
are reported without touching the device."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2401_04576_amd as ia

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ia.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ia_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ia_vote_level", "ia_refine", "ia_find_helices", "ia_estimate", "ia_ctx_create",
              "ia_ctx_destroy", "ia_last_error", "ia_ctx_status"):
        assert n in names


def test_library_exports_every_declared_symbol():
    path = ia.lib_path()
    assert os.path.exists(path), "build libia.so first"
    out = subprocess.check_output(["nm", "-D", "--defined-only", path], text=True)
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    L = ia.load()
    for n in _declared():
        assert hasattr(L, n)


def test_schedule_layout_matches_header():
    # ia_schedule: ia_box (80) + bins (20) + n_refine, top_k (8) + split (20) + v_min,
    # n_helix_max (8) + hitfind_scale (8) + prec[8] (32) + fp32_slack (8) = 184
    assert C.sizeof(ia.Schedule) == 184
    assert ia.HELIX_DTYPE.itemsize == 96 and ia.ESTIMATE_DTYPE.itemsize == 88


def test_host_side_errors_without_device():
    L = ia.load()
    # a null context is rejected before any HIP call
    assert L.ia_vote_level(None, None, 0, None, None, 0, None, 0, None, None) == 1
    assert L.ia_refine(None, None, 0, None, None, 0, 0, None, None, None, None) == 1
    assert L.ia_ctx_create(None, 0, 0) == 1
    s = ia.Schedule.make([0] * 5, [1] * 5, [16] * 5)
    assert ia.Context.scratch_needed(s, 200) > 16 ** 5 * 2
