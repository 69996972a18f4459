"""The ctypes mirrors of the C ABI's structs (paper_2312_06484_amd/airpf.py)
and of the oracle's (oracle/oracle.py) against their headers: a small C program built with the host compiler
from include/airpf.h prints every field's offset and every struct's size,
which must equal what ctypes lays out.  A field added to one side only, or
in another order, fails here before any GPU call could read a shifted
struct."""
import os
import shutil
import subprocess

import pytest

from paper_2312_06484_amd import airpf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("airpf_model", airpf._Model), ("airpf_options", airpf._Options),
         ("airpf_problem", airpf._Problem), ("airpf_trace", airpf._Trace)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a host C compiler")
def test_struct_layouts_match_the_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "airpf.h"', "int main(void) {"]
    for cname, py in PAIRS:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in PAIRS:
        assert got[(cname, "size")] == C_sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a host C compiler")
def test_oracle_struct_layouts_match_its_header(tmp_path):
    from oracle import oracle as orc
    pairs = [("orc_problem", orc._Problem), ("orc_opts", orc._Opts), ("orc_trace", orc._Trace)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "orc.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-I", os.path.join(ROOT, "oracle"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs:
        assert got[(cname, "size")] == C_sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def C_sizeof(py):
    import ctypes
    return ctypes.sizeof(py)
