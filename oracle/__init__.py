"""Oracle: a plain fp64 CPU reference of the Icarus hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and
bench.py's cpu_baseline leg may import, call, link or execute anything
under oracle/.  It shares no code with the HIP library and never imports it.

Modules: units (code units, constants), geometry (stretched/equidistant faces,
Eq. 5), boundary (seeded wind, cone CME Eqs. 1-4, initial state), forest
(block-AMR tree and regrid), solver (two-stage finite-volume step on one patch
or on a block forest, ghost cells, prolongation/restriction/reflux,
refinement flags, point sampling), analysis (arrival time), mlp (the learned
flag network's reference forward/backward).  The numerical core is the C
file oracle.c, loaded through _clib.
"""
from . import units, geometry, boundary, forest, solver, analysis  # noqa: F401
from ._clib import build  # noqa: F401
