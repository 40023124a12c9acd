"""Degenerate inputs through the C ABI.

- An advance over no time, or with a step limit of zero, takes no step: state,
  clock, time and the recorded series stay as they were (the steps an advance
  batch runs past a member's end time take dt = 0 and record no sample).
- A domain of a single block (every face a physical boundary: the inner
  wind / cone-CME boundary, outflow elsewhere) matches the oracle step by
  step, with the CME entering through the inner boundary.
- A block of the smallest shape (4 cells along each direction: two ghost
  layers span a whole block) on a periodic refined box matches the oracle.
- A coarse block whose neighbours along all three axes are refined (reflux
  faces that share edges and a corner, each such cell corrected once per face
  in face order by one thread) matches the oracle step by step.
- A regrid that asks every leaf of the top level to refine leaves the forest
  at the top level."""
import numpy as np
import pytest

from gpu_helpers import rel_err, tiny_wedge
from oracle import forest as fo, solver, units

pytestmark = pytest.mark.gpu


def _ic():
    import paper_2211_12867_amd as ic
    return ic


def test_advance_over_nothing_takes_no_step():
    ic = _ic()
    g, wind, cme, amr = tiny_wedge()
    s = ic.Sim(g, wind, [cme], amr)
    s.step()
    before = (s.blocks(), s.state()[1], s.clock(), s.time(), len(s.timeseries()))
    for dt_s, max_steps in ((0.0, 10), (3600.0, 0)):
        info = s.advance(dt_s, max_steps)
        assert info["steps"] == 1                 # the one step before
        assert s.blocks() == before[0]
        assert np.array_equal(s.state()[1], before[1])
        assert s.clock() == before[2] and s.time() == before[3]
        assert len(s.timeseries()) == before[4]
    s.close()


def test_single_block_domain_matches_the_oracle():
    ic = _ic()
    g, wind, cme, amr = tiny_wedge()
    g = dict(g, x1=(0.35, 120.0, 90.0), n=(12, 12, 12), block=(12, 12, 12))
    cme = dict(cme, lon_deg=45.0, t_start_s=0.0)
    ora = solver.Solver(g, wind, cme, amr)
    gpu = ic.Sim(g, wind, [cme], amr)
    assert len(gpu.blocks()) == 1
    gpu.set_state(*ora.state(), 0.0)
    for n in range(12):
        info = gpu.step()
        dt = ora.step()
        assert abs(info["dt_s"] / units.T0 - dt) <= 1e-12 * dt
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-12 * (n + 1), (n, e)
    gpu.close()


def test_smallest_block_shape_on_a_refined_box():
    ic = _ic()
    box = dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 1.0, 1.0), n=(8, 8, 8), block=(4, 4, 4),
               periodic=(True, True, True), max_level=2, gamma=1.5, cfl=0.4)
    ora = solver.Solver(box, initial="zero", amr=dict(buffer_blocks=0))
    g = np.random.default_rng(21)
    for leaf in ora.forest.leaves:
        x = [ora.centres(leaf, d) for d in range(3)]
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        W = np.zeros((8,) + X.shape)
        base = [1.0, 0.2, -0.1, 0.15, 1.0, 0.3, 0.2, -0.1]
        for v in range(8):
            k = g.integers(1, 3, size=3)
            W[v] = base[v] + (0.1 if v in (0, 4) else 0.2) * np.sin(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z)
                                                                  + g.uniform(0, 2 * np.pi))
        from oracle import boundary
        ora.U[leaf] = boundary.prims_to_cons(W, 1.5)
    ora.regrid({b: (fo.REFINE if b == (1, 0, 0, 0) else fo.KEEP) for b in ora.forest.leaves}, buffer_blocks=0)
    gpu = ic.Sim(box, amr=dict(buffer_blocks=0))
    gpu.set_state(*ora.state(), 0.0)
    assert max(b[0] for b in gpu.blocks()) == 2
    for n in range(6):
        gpu.step()
        ora.step()
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-12 * (n + 1), (n, e)
    gpu.close()


def _smooth_box_state(ora, seed):
    from oracle import boundary
    g = np.random.default_rng(seed)
    for leaf in ora.forest.leaves:
        x = [ora.centres(leaf, d) for d in range(3)]
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        W = np.zeros((8,) + X.shape)
        base = [1.0, 0.2, -0.1, 0.15, 1.0, 0.3, 0.2, -0.1]
        for v in range(8):
            k = g.integers(1, 3, size=3)
            W[v] = base[v] + (0.1 if v in (0, 4) else 0.2) * np.sin(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z)
                                                                  + g.uniform(0, 2 * np.pi))
        ora.U[leaf] = boundary.prims_to_cons(W, 1.5)


def test_reflux_faces_meeting_at_edges_and_a_corner():
    ic = _ic()
    box = dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 1.0, 1.0), n=(16, 16, 16), block=(4, 4, 4),
               periodic=(True, True, True), max_level=2, gamma=1.5, cfl=0.4)
    ora = solver.Solver(box, initial="zero", amr=dict(buffer_blocks=0))
    _smooth_box_state(ora, 33)
    # the coarse block (1, 1, 1) keeps level 1; its -x, -y and -z neighbours refine
    fine = {(1, 0, 1, 1), (1, 1, 0, 1), (1, 1, 1, 0)}
    ora.regrid({b: (fo.REFINE if b in fine else fo.KEEP) for b in ora.forest.leaves}, buffer_blocks=0)
    gpu = ic.Sim(box, amr=dict(buffer_blocks=0), max_blocks=256)
    gpu.set_state(*ora.state(), 0.0)
    assert sum(1 for b in gpu.blocks() if b[0] == 2) == 24
    for n in range(6):
        gpu.step()
        ora.step()
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-12 * (n + 1), (n, e)
    gpu.close()


def test_refining_the_top_level_keeps_the_forest():
    ic = _ic()
    box = dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 1.0, 1.0), n=(8, 8, 8), block=(8, 8, 8),
               periodic=(True, True, True), max_level=2, gamma=1.5, cfl=0.4)
    s = ic.Sim(box, amr=dict(buffer_blocks=0), max_blocks=64)
    s.regrid([np.ones(len(s.blocks()), np.int8)])          # level 1 -> 2
    top = s.blocks()
    assert len(top) == 8 and all(b[0] == 2 for b in top)
    U = s.state()[1]
    s.regrid([np.ones(len(top), np.int8)])                  # nothing above the top level
    assert s.blocks() == top
    assert np.array_equal(s.state()[1], U)
    s.close()
