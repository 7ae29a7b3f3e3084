"""The C-ABI library loads and exports every symbol include/d2d.h declares (CPU only)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "d2d.h")
LIB = os.path.join(ROOT, "paper_0707_0159_amd", "libd2d.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(d2d_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("d2d_ctx_create", "d2d_block_import", "d2d_sb_create", "d2d_hv", "d2d_lanczos",
                 "d2d_density_matrix", "d2d_batch_lanczos"):
        assert must in names


def test_library_exports_every_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libd2d.so is not built: run python -m paper_0707_0159_amd.build")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(d2d_[a-z0-9_]+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_loads_and_reports_errors():
    from paper_0707_0159_amd import d2d
    lib = d2d.load()
    for n in declared():
        assert hasattr(lib, n)
    assert set(d2d.EXPORTED) == set(declared())
    assert "gfx950" in d2d.d2d_version()
    # error path without a GPU: NULL out pointer is rejected before any device call
    assert lib.d2d_ctx_create(0, None, 0, None) == d2d.D2D_EINVAL
    assert "NULL" in d2d.d2d_last_error()


def test_splitmix64_known_answers():
    """The seeded start-vector generator against the SplitMix64 reference
    outputs for seed 1234567 (the published test vector of the generator)."""
    import numpy as np
    import workloads as W
    assert [int(x) for x in W.splitmix64(1234567, 5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
        16408922859458223821]
    z = W.splitmix_normal(200000, 7)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


def test_lanczos_opts_layout(tmp_path):
    """The binding's options and stats structs have the layout a C compiler
    gives the header's: every field offset and the size, printed by a small C
    program built with gcc against include/d2d.h."""
    import ctypes as C
    import shutil
    import subprocess
    from paper_0707_0159_amd import d2d
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"d2d_lanczos_opts": d2d.d2d_lanczos_opts, "d2d_lanczos_stats": d2d.d2d_lanczos_stats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "d2d.h"', "int main(void) {"]
    for name, py in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, py in structs.items():
        assert got[(name, "size")] == C.sizeof(py), name
        for f, _ in py._fields_:
            assert got[(name, f)] == getattr(py, f).offset, (name, f)
