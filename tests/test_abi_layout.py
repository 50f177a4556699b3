"""The ctypes binding lays out every struct of include/seraph.h exactly as the
C compiler does: size and the offset of every field, read from a small C
program compiled against the header."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = ["sr_pvu_diagram", "sr_run_params", "sr_run_stats", "sr_sweep_record", "sr_graph_info",
           "sr_page_view", "sr_instance", "sr_batch_stats", "sr_server_stats"]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    import paper_1806_00762_amd as sr
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "seraph.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(sr, name, None)
        if cls is None:
            continue
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            field = f[0].rstrip("_") if f[0] == "pass_" else f[0]
            lines.append(f'  printf("{name} {f[0]} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    table = {}
    for line in out.splitlines():
        s, f, v = line.split()
        table[(s, f)] = int(v)
    return sr, table


@pytest.mark.parametrize("name", STRUCTS)
def test_struct_layout_matches_header(c_layout, name):
    sr, table = c_layout
    cls = getattr(sr, name, None)
    assert cls is not None, f"binding has no {name}"
    assert ctypes.sizeof(cls) == table[(name, "size")], f"{name}: size differs"
    for f in cls._fields_:
        assert getattr(cls, f[0]).offset == table[(name, f[0])], f"{name}.{f[0]}: offset differs"
