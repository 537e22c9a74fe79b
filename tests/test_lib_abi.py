"""CPU checks of the C-ABI library: it is built, loads, and exports every symbol include/nlf.h
declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1410_3584_amd", "libnlf.so")
HEADER = os.path.join(ROOT, "include", "nlf.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nlf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnlf.so is not built (run `python -m paper_1410_3584_amd.build`)")
    return ctypes.CDLL(LIB)


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ["nlf_plan_create", "nlf_potential", "nlf_type2", "nlf_type1", "nlf_ground_state", "nlf_evolve"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_export_list_matches_header():
    from paper_1410_3584_amd import nlf
    assert sorted(nlf.EXPORTS) == declared_functions()


def test_status_strings(lib):
    lib.nlf_strerror.restype = ctypes.c_char_p
    lib.nlf_version.restype = ctypes.c_char_p
    assert lib.nlf_strerror(0) == b"ok"
    assert lib.nlf_strerror(-5).startswith(b"iteration cap")
    assert b"gfx950" in lib.nlf_version()


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the sizes and field offsets the C compiler gives the
    declarations in include/nlf.h (compiled here with gcc)."""
    import subprocess
    from paper_1410_3584_amd import nlf
    structs = {"nlf_box": nlf.Box, "nlf_opts": nlf.Opts, "nlf_plan_info": nlf.PlanInfo,
               "nlf_phys": nlf.Phys, "nlf_gf_opts": nlf.GfOpts, "nlf_gs_stats": nlf.GsStats,
               "nlf_ts_opts": nlf.TsOpts}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "nlf.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
