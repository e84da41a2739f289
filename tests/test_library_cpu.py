"""CPU-only checks of the HIP library: it loads, exports every symbol the C
header declares, its host-side helpers match the oracle, and argument errors
are reported without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "fl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1503_03635_amd import _lib
    L = _lib.lib()
    syms = _header_symbols()
    assert "fl_solve" in syms and "fl_ads_build" in syms and "fl_solve_batch" in syms
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(_lib.SIGNATURES), "binding and header disagree"


def test_host_ranks_match_oracle():
    import oracle as O
    from paper_1503_03635_amd import priority_of, rank_of
    for seed in (0, 1, 99, 2 ** 63 + 5):
        r, p = O.ranks(3000, seed)
        assert all(rank_of(i, seed) == r[i] for i in range(0, 3000, 7))
        assert all(priority_of(i, seed) == p[i] for i in range(0, 3000, 7))


def test_strerror_and_param_errors_without_gpu():
    from paper_1503_03635_amd import _lib
    L = _lib.lib()
    for code in range(7):
        assert L.fl_strerror(code)
    prob = _lib.FlProblem(0, 0, None, None, None, None, None)
    prm = _lib.FlParams(16, 1, 0.1, 0)
    res = _lib.FlResult()
    # n = 0 and k = 0 are rejected before any device call
    assert L.fl_solve(C.byref(prob), C.byref(prm), C.byref(res), None) == _lib.FL_EINVAL
    prob.n = 10
    prm.k = 0
    assert L.fl_solve(C.byref(prob), C.byref(prm), C.byref(res), None) == _lib.FL_EINVAL
    assert L.fl_solve(None, C.byref(prm), C.byref(res), None) == _lib.FL_EINVAL
    assert res.n_open == 0


def test_binding_structs_match_the_header(tmp_path):
    """Every field of the ctypes structs sits at the offset the C compiler
    gives it from include/fl.h (a mismatch would corrupt results silently)."""
    import subprocess
    from paper_1503_03635_amd import _lib
    structs = {"fl_problem": _lib.FlProblem, "fl_params": _lib.FlParams, "fl_stats": _lib.FlStats,
               "fl_result": _lib.FlResult}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "fl.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
