"""The C ABI library loads on any host and exports every entry point include/wq.h declares
(no compute calls: those need a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_29334_amd", "libwq.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        subprocess.run(["python", os.path.join(ROOT, "paper_2605_29334_amd", "build.py")], check=True)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("build_points", "solve_weights", "assemble_mass", "assemble_stiffness", "assemble_biharmonic",
              "wq_mesh_create", "wq_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_2605_29334_amd.wq as W
    assert set(W.exported_symbols()) <= set(declared_functions())


def test_strerror_is_host_only(lib):
    lib.wq_strerror.restype = ctypes.c_char_p
    assert lib.wq_strerror(-3).startswith(b"ill-posed")


def test_side_streams_setting_is_host_only(lib):
    """wq_set_side_streams only records the count (1..8) for later calls: no device work."""
    lib.wq_set_side_streams.argtypes = [ctypes.c_int32]
    lib.wq_set_side_streams.restype = ctypes.c_int
    assert lib.wq_set_side_streams(0) != 0 and lib.wq_set_side_streams(9) != 0
    try:
        assert lib.wq_set_side_streams(1) == 0 and lib.wq_set_side_streams(8) == 0
    finally:
        assert lib.wq_set_side_streams(4) == 0


def test_struct_layouts_match_the_binding(tmp_path):
    """Sizes and field offsets of the ABI structs, as a C compiler lays them out from
    include/wq.h, equal the ctypes mirrors of the binding."""
    import paper_2605_29334_amd.wq as W
    structs = {"wq_mesh_desc": W.MeshDesc, "wq_timing": W.Timing, "wq_solve_report": W.SolveReport,
               "wq_conductivity": W.Conductivity, "wq_heat_params": W.HeatParams, "wq_heat_report": W.HeatReport,
               "wq_request": W.Request, "wq_result": W.Result}
    rename = {"lam": "lambda"}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "wq.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {rename.get(f, f)}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
