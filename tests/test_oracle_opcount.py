"""Operation count of the oracle's spatial operator (measurement of the oracle,
CPU only): oracle/opcount.cpp compiles the oracle's C core with a counting
floating-point type.  Checked here: it builds and runs on a physical state,
the pointwise pieces have the counts their formulas give (primitive recovery:
3 divisions and 17 adds/multiplies; MC slope: 3 divisions, 6 adds, 4
multiplies), and the operator's count per cell lies between the count of its
faces' Rusanov fluxes alone and a generous bound."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(tmp_path):
    exe = str(tmp_path / "opcount")
    subprocess.check_call(["g++", "-O1", "-std=c++17", os.path.join(ROOT, "oracle", "opcount.cpp"), "-o", exe])
    out = subprocess.check_output([exe], text=True)
    rows = {}
    for line in out.splitlines():
        parts = line.split()
        if len(parts) == 2:
            rows[parts[0]] = float(parts[1])
        else:
            rows[parts[0]] = {parts[q]: float(parts[q + 1]) for q in range(1, len(parts), 2)}
    return rows


def test_opcount_builds_and_counts(tmp_path):
    r = _run(tmp_path)
    assert r["bad"] == 0
    assert r["prim"]["div"] == 3 and r["prim"]["add"] + r["prim"]["mul"] == 17
    assert r["mc_slope"] == dict(add=6, mul=4, div=3, sqrt=0, trig=0, cmp=4, flops=13)
    assert r["fast_speed"]["sqrt"] == 2 and r["rusanov"]["sqrt"] == 4
    faces_per_cell = r["faces"] / r["cells"]
    rhs = r["rhs_per_cell"]["flops"]
    assert faces_per_cell * r["rusanov"]["flops"] < rhs < 4000
    print({k: v for k, v in r.items()})
