"""The ctypes mirrors of the C-ABI structures match the C header's layout:
sizes and field offsets as a C compiler lays them out (gcc on include/bns.h)."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ("bns_options", "bns_ci_test", "bns_depth_stats")


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    from paper_2212_04259_amd import _lib
    d = tmp_path_factory.mktemp("layout")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bns.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append(f'    printf("{s} sizeof %zu\\n", sizeof({s}));')
        for name, _ in getattr(_lib, s)._fields_:
            lines.append(f'    printf("{s} {name} %zu\\n", offsetof({s}, {name}));')
    lines += ["    return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([gcc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        s, name, val = line.split()
        layout[(s, name)] = int(val)
    return layout


@pytest.mark.parametrize("struct", STRUCTS)
def test_struct_layout_matches_header(c_layout, struct):
    from paper_2212_04259_amd import _lib
    cls = getattr(_lib, struct)
    assert ctypes.sizeof(cls) == c_layout[(struct, "sizeof")]
    for name, _ in cls._fields_:
        assert getattr(cls, name).offset == c_layout[(struct, name)], name
