"""Host-side checks of the library (no GPU): the shared library loads and
exports every entry point of include/dp.h, its argument validation, and its
host colouring equals the oracle's bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2106_01275_amd as dp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "dp.h")).read()
    declared = set(re.findall(r"^\s*(?:dp_status|void|const char \*)\s*\*?\s*(dp_\w+)\s*\(", hdr, re.M))
    assert declared == set(dp.EXPORTS)
    L = ctypes.CDLL(dp.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets of the C structs."""
    src = tmp_path / "sz.c"
    fields = {"dp_probe_spec": ["colors_dev", "seed", "dilute"], "dp_operator": ["m2", "links"],
              "dp_solve_opts": ["reliable_delta", "profile"], "dp_solve_stats": ["max_true_resid", "stencil_bytes", "seconds", "stencil_bytes_all"],
              "dp_trace_result": ["per_rhs", "solve"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dp.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("%zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    import subprocess
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    mirrors = {"dp_probe_spec": dp.ProbeSpec, "dp_operator": dp.Operator, "dp_solve_opts": dp.SolveOpts,
               "dp_solve_stats": dp.SolveStats, "dp_trace_result": dp.TraceResult}
    want = []
    for st, fs in fields.items():
        cls = mirrors[st]
        want.append(ctypes.sizeof(cls))
        for f in fs:
            want.append(getattr(cls, "stderr_" if f == "stderr" else f).offset)
    assert got == want


@pytest.mark.parametrize("dims,p,ks,order", [
    ((4, 4, 4, 4), 1, 2, "natural"), ((4, 4, 4, 4), 1, 2, "redblack"),
    ((8, 8, 8, 8), 2, 4, "natural"), ((8, 8, 8, 8), 2, 4, "redblack"), ((8, 8, 8, 8), 2, 4, "best"),
    ((5, 3, 4, 2), 3, 1, "natural"), ((6, 6, 4, 4), 1, [1, 2, 3], "natural"),
    ((16, 8, 8, 8), 2, 3, "best"), ((32, 1, 1, 1), 0, 3, "natural"), ((3, 3, 3, 3), 0, 5, "natural"),
    ((12, 10, 6, 8), 3, 4, "best"),
])
def test_coloring_bit_exact_with_oracle(dims, p, ks, order):
    col, n, used = dp.build_coloring(dims, p, ks, order)
    okind = {"natural": oracle.NATURAL, "redblack": oracle.REDBLACK, "best": oracle.BEST}[order]
    if np.isscalar(ks):
        want, wn, wused = oracle.coloring(dims, p, ks, okind)
        assert n == wn and np.array_equal(col, want)
        assert {"natural": oracle.NATURAL, "redblack": oracle.REDBLACK}[used] == wused
    else:
        want, wn = oracle.coloring_nested(dims, p, ks, okind)
        assert np.array_equal(n, wn) and np.array_equal(col, want)


@pytest.mark.slow
def test_coloring_nested_16_bit_exact():
    """The 16^4 nested levels (p = 4, distances 1, 2, 4, 8): 3/5/16/960 colours."""
    col, n, _ = dp.build_coloring((16, 16, 16, 16), 4, [1, 2, 4, 8], "natural")
    assert list(n) == [3, 5, 16, 960]
    want, wn = oracle.coloring_nested((16, 16, 16, 16), 4, [1, 2, 4, 8])
    assert np.array_equal(col, want)


def test_coloring_rejects_bad_arguments():
    with pytest.raises(dp.DPError):
        dp.build_coloring((4, 4, 0, 4), 1, 2)
    with pytest.raises(dp.DPError):
        dp.build_coloring((4, 4, 4, 4), -1, 2)
    with pytest.raises(dp.DPError):
        dp.build_coloring((4, 4, 4, 4), 1, [2, 2])
