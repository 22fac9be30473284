"""The binding's ctypes structures against the C header: a small C program
compiled against include/msp.h prints sizeof and offsetof of every field the
binding declares, and both must agree (a field added on one side only shifts
every later field)."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["msp_csr", "msp_symmap", "msp_copies", "msp_opts", "msp_stats", "msp_faces"]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_ctypes_structures_match_the_header(tmp_path):
    from paper_2407_05930_amd import _lib
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "msp.h"', "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'    printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in getattr(_lib, name)._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            s, f, v = ln.split()
            got[(s, f)] = int(v)
    for name in STRUCTS:
        cls = getattr(_lib, name)
        assert got[(name, "sizeof")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
