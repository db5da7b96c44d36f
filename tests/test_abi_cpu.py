"""The C-ABI library loads and exports every entry point include/svt.h
declares (no GPU needed: nothing here launches device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svt.h")
LIB = os.path.join(ROOT, "paper_1311_0380_amd", "libsvt.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svt_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("svt_create", "svt_destroy", "svt_load_constants", "svt_fit_events",
                 "svt_result", "svt_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libsvt.so not built: run __graft_entry__.build()")
    import torch  # noqa: F401  (one HIP runtime per process: torch's)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1311_0380_amd import svt
    assert sorted(svt.SIGNATURES) == declared() or set(declared()) <= set(svt.SIGNATURES)


def test_status_strings():
    from paper_1311_0380_amd import svt
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert svt.svt_status_string(code).startswith("SVT_")


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding mirrors has the size and field offsets the
    C compiler gives it from include/svt.h (host compiler, no GPU)."""
    import shutil
    import subprocess
    from paper_1311_0380_amd import svt
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"svt_event_batch": svt.svt_event_batch, "svt_results": svt.svt_results,
               "svt_summary": svt.svt_summary, "svt_tuning": svt.svt_tuning,
               "svt_device_info": svt.svt_device_info,
               "svt_shadow_tracks": svt.svt_shadow_tracks, "svt_pass_list": svt.svt_pass_list,
               "svt_unpack_out": svt.svt_unpack_out}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "svt.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
