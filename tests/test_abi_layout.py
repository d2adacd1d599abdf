"""The Python binding's ctypes structures match include/fmmlu.h field for field: a small C
program built with the host compiler prints the size of fmmlu_opts and fmmlu_info and the
offset of every field the binding declares, and they must equal ctypes' layout (a field
added to the header and not to the binding, or in another order, shifts everything after
it)."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2201_07325_amd as fm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_structures_match_the_header(tmp_path):
    structs = {"fmmlu_opts": fm.Opts, "fmmlu_info": fm.Info}
    lines = ["#include <stddef.h>", "#include <stdio.h>", "#include \"fmmlu.h\"", "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            cname, key, val = ln.split()
            got[(cname, key)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)

