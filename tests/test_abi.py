"""The C-ABI library loads on the CPU and exports every symbol the header
declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crowdsplat.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:cs_status|void|const char\*)\s+(cs_\w+)\s*\(", text, re.M)))


def test_header_declares_the_five_entry_points():
    names = _declared()
    for n in ["cs_upload_templates", "cs_skin_instances", "cs_select_lod", "cs_render_frame",
              "cs_render_backward"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2501_17792_amd import crowdsplat

    if not os.path.exists(crowdsplat.LIB_PATH):
        pytest.fail("libcrowdsplat.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(crowdsplat.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(crowdsplat.EXPORTS) == _declared()
    crowdsplat.load_library()
    assert b"gfx950" in crowdsplat._lib.cs_version()


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """ctypes mirrors of the header's structs have the C compiler's sizes and
    field offsets."""
    import shutil
    import subprocess

    from paper_2501_17792_amd import crowdsplat as cs

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"cs_options": cs.CsOptions, "cs_template_desc": cs.CsTemplateDesc,
               "cs_camera": cs.CsCamera, "cs_lod_params": cs.CsLodParams,
               "cs_frame_stats": cs.CsFrameStats, "cs_template_grads": cs.CsTemplateGrads,
               "cs_mlp": cs.CsMlp, "cs_memory_stats": cs.CsMemoryStats,
               "cs_pose_net": cs.CsPoseNet}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "crowdsplat.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
    assert cs.INSTANCE_DTYPE.itemsize == 16


def test_null_context_calls_return_invalid():
    from paper_2501_17792_amd import crowdsplat as cs

    lib = cs.load_library()
    assert lib.cs_upload_templates(None, None, 0, 0) == cs.CS_ERR_INVALID
    assert lib.cs_render_frame(None, None, None, None) == cs.CS_ERR_INVALID
    assert lib.cs_frame_launch(None) == cs.CS_ERR_INVALID
    lib.cs_destroy(None)


def test_header_constants_match_the_binding():
    """Every integer constant of the header that the binding mirrors (LoD
    modes, debug buffers, sort and launch options, limits) has the header's
    value, so a new mode or buffer cannot drift between the two."""
    from paper_2501_17792_amd import crowdsplat as cs

    text = open(HEADER).read()
    consts = {}
    for name, val in re.findall(r"^#define\s+(CS_\w+)\s+(\(1 << \d+\)|-?\d+)\b", text, re.M):
        consts[name] = 1 << int(val[6:-1]) if val.startswith("(") else int(val)
    checked = 0
    for name, val in consts.items():
        if name.startswith("CS_BUF_"):
            assert cs.BUF[name[len("CS_BUF_"):]] == val, name
            checked += 1
        elif hasattr(cs, name):
            assert getattr(cs, name) == val, name
            checked += 1
    assert "CS_LOD_BUDGET_VISIBLE" in consts and cs.CS_LOD_BUDGET_VISIBLE == consts["CS_LOD_BUDGET_VISIBLE"]
    assert len(cs.BUF) == sum(1 for n in consts if n.startswith("CS_BUF_"))
    assert checked >= 20
