"""The ctypes mirrors of the problem and option structures in the binding
have the C layout of include/attn.h: a small C program compiled against the
header prints the size and every field offset, and the binding must agree."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["attn_problem", "attn_solver_opts", "attn_sweep_opts", "attn_batch_opts", "attn_de_opts"]


def test_struct_layout_matches_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    from paper_2507_21236_amd import _lib
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "attn.h"', "int main(void) {"]
    for name in STRUCTS:
        src.append(f'  printf("{name} __size__ %zu\\n", sizeof({name}));')
        for field, _ in getattr(_lib, name)._fields_:
            src.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    src += ["  return 0;", "}"]
    c_file = tmp_path / "layout.c"
    c_file.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(c_file), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c_layout = {}
    for line in out:
        if line:
            name, field, value = line.split()
            c_layout[(name, field)] = int(value)
    for name in STRUCTS:
        py = getattr(_lib, name)
        assert c_layout[(name, "__size__")] == ctypes.sizeof(py), name
        for field, _ in py._fields_:
            assert c_layout[(name, field)] == getattr(py, field).offset, (name, field)
