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


def _c_layout(tmp_path):
    """sizeof and field offsets of the ABI structs as the C compiler lays them out"""
    src = tmp_path / "layout.c"
    fields = {"ia_schedule": ["range", "bins", "n_refine", "top_k", "split", "v_min", "n_helix_max",
                              "hitfind_scale", "prec", "fp32_slack", "mode", "forward", "move_level", "wdrop", "hitsel",
                              "lbins", "disk"],
              "ia_helix": ["p", "err", "ref", "votes", "n_assigned", "n_argmax", "status"],
              "ia_estimate_t": ["p", "err", "vmax", "n_argmax"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ia.h"', "int main(void) {"]
    for t, fs in fields.items():
        lines.append(f'  printf("{t} sizeof %zu\\n", sizeof({t}));')
        for f in fs:
            lines.append(f'  printf("{t} {f} %zu\\n", offsetof({t}, {f}));')
    lines.append("  return 0;\n}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        t, f, v = line.split()
        out[(t, f)] = int(v)
    return out


def test_struct_layouts_match_header(tmp_path):
    """ctypes / numpy layouts of the binding equal the C compiler's for ia.h"""
    lay = _c_layout(tmp_path)
    assert C.sizeof(ia.Schedule) == lay[("ia_schedule", "sizeof")]
    for name, _ in ia.Schedule._fields_:
        assert getattr(ia.Schedule, name).offset == lay[("ia_schedule", name)], name
    for dt, t in ((ia.HELIX_DTYPE, "ia_helix"), (ia.ESTIMATE_DTYPE, "ia_estimate_t")):
        assert dt.itemsize == lay[(t, "sizeof")]
        for name in dt.names:
            assert dt.fields[name][1] == lay[(t, name)], (t, name)


def test_host_side_errors_without_device():
    L = ia.load()
    # a null context is rejected before any HIP call
    assert L.ia_vote_level(None, None, 0, None, None, 0, None, 0, None, None) == 1
    assert L.ia_refine(None, None, 0, None, None, 0, 0, None, None, None, None) == 1
    assert L.ia_ctx_create(None, 0, 0) == 1
    s = ia.Schedule.make([0] * 5, [1] * 5, [16] * 5)
    assert ia.Context.scratch_needed(s, 200) > 16 ** 5 * 2
