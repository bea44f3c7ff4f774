"""The C-ABI library loads on the CPU host and exports every symbol include/rpb.h declares."""
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rpb.h")
LIB = os.path.join(ROOT, "paper_1612_00474_amd", "librpb.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char|double)\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("rpb_mobility_matvec", "lanczos_sqrt_apply", "rfd_drift", "sab_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librpb.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librpb.so not built (run __graft_entry__.build())")
def test_binding_loads_and_matches_header():
    from paper_1612_00474_amd import _lib
    lib = _lib.load()
    assert sorted(_lib.EXPORTS) == declared_functions()
    for name in _lib.EXPORTS:
        assert hasattr(lib, name)
    assert lib.rpb_version().decode().startswith("librpb")


def test_ctypes_structs_match_the_header_layout(tmp_path):
    # every field offset and struct size of the binding's mirrors, against gcc on rpb.h
    import ctypes as C
    from paper_1612_00474_amd import _lib
    structs = {"rpb_params": _lib.RpbParams, "rpb_sab_config": _lib.RpbSabConfig,
               "rpb_shape": _lib.RpbShape, "rpb_tuning": _lib.RpbTuning,
               "rpb_sab_state": _lib.RpbSabState}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rpb.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        cname, what, value = line.split()
        py = structs[cname]
        expect = C.sizeof(py) if what == "size" else getattr(py, what).offset
        assert int(value) == expect, (cname, what)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in structs.values())
