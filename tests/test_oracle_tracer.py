"""Pins of the oracle's CME density tracer and the tracer / combined
refinement criteria (paper Sect. 3.1: a density tracer injected with the CME,
the grid refined where it is non-zero; Sect. 3.3: combined with the shock
criterion inside the Earth windows).

- The tracer is passive: the eight MHD variables are bit-identical with and
  without it.
- With s = 1 everywhere the tracer equation is the continuity equation: rho s
  stays equal to rho bit for bit (the flux form and the shared c_max).
- A smooth tracer profile in a uniform flow translates with the flow:
  second-order convergence to s(x - v t), and the total rho s is conserved.
- At the inner boundary the cone CME brings s = 1 and the wind s = 0.
- Tracer criterion: REFINE where some cell has s above tracer_refine, with no
  windows; the combined criterion ORs it with the shock condition inside the
  windows.
"""
import math

import numpy as np
import pytest

from oracle import boundary, forest as fo, solver
from synthetic import as_dict, workload

GAMMA = 1.5


def _box(n, L=(1.0, 0.25, 0.25)):
    return dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=L, n=n, block=n, periodic=(True, True, True),
                gamma=GAMMA, cfl=0.4)


def _smooth(s, seed, with_tracer):
    nk, nj, ni = s.U.shape[1:]
    rng = np.random.default_rng(seed)
    x = (np.arange(ni) + 0.5) / ni
    W = np.zeros((9 if with_tracer else 8, nk, nj, ni))
    W[0] = 1.0 + 0.2 * np.sin(2 * math.pi * x)
    W[1] = 0.6 + 0.1 * np.cos(2 * math.pi * x)
    W[2] = 0.05
    W[4] = 1.0 + 0.1 * np.sin(4 * math.pi * x)
    W[5] = 0.4
    W[6] = 0.2 * np.cos(2 * math.pi * x)
    if with_tracer:
        W[8] = 0.5 + 0.5 * np.sin(2 * math.pi * x + rng.uniform(0, 1))
    return W


def test_tracer_is_passive():
    a = solver.PatchSolver(_box((32, 2, 2)), initial="zero")
    b = solver.PatchSolver(_box((32, 2, 2)), initial="zero", tracer=True)
    W = _smooth(b, 1, True)
    b.U = boundary.prims_to_cons(W, GAMMA)
    a.U = boundary.prims_to_cons(W[:8], GAMMA)
    for _ in range(20):
        a.step()
        b.step()
    assert np.array_equal(a.U, b.U[:8])


def test_uniform_fraction_tracer_is_the_density():
    s = solver.PatchSolver(_box((32, 2, 2)), initial="zero", tracer=True)
    W = _smooth(s, 2, True)
    W[8] = 1.0
    s.U = boundary.prims_to_cons(W, GAMMA)
    for _ in range(20):
        s.step()
        assert np.array_equal(s.U[8], s.U[0])


def _advect(N, t_end=0.25):
    s = solver.PatchSolver(_box((N, 1, 1), L=(1.0, 1.0 / N, 1.0 / N)), initial="zero", tracer=True)
    x = (np.arange(N) + 0.5) / N
    W = np.zeros((9, 1, 1, N))
    W[0] = 1.0
    W[1] = 0.8
    W[4] = 1.0
    W[5] = 0.3
    W[8] = 0.5 + 0.4 * np.sin(2 * math.pi * x)
    s.U = boundary.prims_to_cons(W, GAMMA)
    tot0 = s.U[8].sum()
    t = 0.0
    while t < t_end - 1e-14:
        h = min(s.cfl_dt(), t_end - t)
        s.step(h)
        t += h
    exact = 0.5 + 0.4 * np.sin(2 * math.pi * (x - 0.8 * t_end))
    assert abs(s.U[8].sum() - tot0) <= 1e-13 * tot0
    assert np.all(s.U[0] == 1.0)            # the carrier flow stays uniform
    return np.abs(s.U[8, 0, 0] / s.U[0, 0, 0] - exact).mean()


def test_smooth_tracer_translates_at_second_order():
    e = [_advect(N) for N in (32, 64, 128)]
    assert math.log(e[1] / e[2], 2.0) >= 1.8 and math.log(e[0] / e[1], 2.0) >= 1.6, e


def test_inner_boundary_brings_cme_material():
    w = workload("tiny_wedge")
    g, wind, cme, amr = as_dict(w.grid), as_dict(w.wind), as_dict(w.cmes[0]), as_dict(w.amr)
    s = solver.Solver(g, wind, cme, amr, tracer=True)
    assert all(np.all(u[8] == 0.0) for u in s.U.values())
    for _ in range(15):
        s.step()
    G = s.ghosted(s.U, s.t)
    inner = [b for b in s.forest.leaves if b[1] == 0]
    fr = []
    for b in inner:
        th = s.centres(b, 1)[None, :, None]
        ph = s.centres(b, 2)[:, None, None]
        m = boundary.cme_mask(cme, th + 0 * ph, ph + 0 * th, s.r_in, s.t)[:, :, 0]
        sg = G[b][8, 2:-2, 2:-2, 0] / G[b][0, 2:-2, 2:-2, 0]       # ghost layer next to r_in
        assert np.all(sg[m] == 1.0) and np.all(sg[~m] == 0.0)
        fr.append(s.U[b][8, :, :, 0] / s.U[b][0, :, :, 0])
    fr = np.concatenate([f.ravel() for f in fr])
    assert fr.max() > 0.5 and fr.min() >= -1e-9       # at most tiny undershoots of the limited scheme


def test_tracer_and_combined_criteria():
    g = dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 1.0, 1.0), n=(8, 8, 8), block=(4, 4, 4),
             periodic=(True, True, True), max_level=2, gamma=GAMMA)
    base = dict(use_windows=False, tracer_refine=0.01, tracer_coarsen=0.00125)
    s = solver.Solver(g, initial="zero", tracer=True, amr=dict(base, criterion="tracer"))
    for leaf in s.forest.leaves:
        W = np.zeros((9,) + s.B[::-1])
        W[0] = 1.0
        W[4] = 1.0
        W[8] = 0.0
        if leaf == (1, 1, 0, 1):
            W[8, 1, 2, 3] = 0.02          # one cell above the refine threshold
        if leaf == (1, 0, 1, 0):
            W[8, 0, 0, 0] = 0.005         # above the coarsen threshold only
        s.U[leaf] = boundary.prims_to_cons(W, GAMMA)
    f = s.flags()
    assert f[(1, 1, 0, 1)] == fo.REFINE
    assert all(v == fo.KEEP for b, v in f.items() if b != (1, 1, 0, 1))    # level 1 never coarsens
    s.regrid(f, buffer_blocks=0)
    f2 = s.flags()
    kids = [b for b in s.forest.leaves if b[0] == 2]
    assert len(kids) == 8
    hot_kid = [b for b in kids if np.any(s.U[b][8] / s.U[b][0] > 0.01)]
    assert all(f2[b] == (fo.KEEP if b in hot_kid or np.any(s.U[b][8] / s.U[b][0] > 0.00125) else fo.COARSEN)
               for b in kids)
    # the shock criterion ignores the tracer; the combined one ORs it in
    s.amr["criterion"] = "shock"
    assert all(v != fo.REFINE for v in s.flags().values())
    s.amr["criterion"] = "combined"
    assert s.flags() == f2
