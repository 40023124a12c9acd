"""Parabolic div B cleaning through the C ABI against the oracle (paper
Sect. 2.1 applies parabolic cleaning in every run): a periodic box of blocks
with a non-solenoidal field (D read across same-level block faces), a
refined box (no gradient across the level change), the cone-CME wedge
(inner and outflow boundaries) with both time schemes.  Bars: <= 1e-12 per
step, <= 1e-10 over 20 steps."""
import math

import numpy as np
import pytest

from gpu_helpers import rel_err, tiny_wedge
from oracle import _clib, boundary, forest as fo, solver, units
from synthetic import smooth_modes

pytestmark = pytest.mark.gpu


def _ic():
    import paper_2211_12867_amd as ic
    return ic


def _box(levels=1):
    return dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 1.0, 0.5), n=(16, 16, 8), block=(8, 8, 8),
                periodic=(True, True, True), max_level=levels, gamma=1.5, cfl=0.4)


def _noisy_field(s, seed):
    for leaf in s.forest.leaves:
        x = [s.centres(leaf, d) for d in range(3)]
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        W = np.zeros((8,) + X.shape)
        base = [1.0, 0.05, -0.05, 0.02, 1.0, 0.3, 0.2, -0.1]
        for v in range(8):
            ks, amps, ph = smooth_modes(seed + v, 3, 0.15 if v in (0, 4) else 0.25)
            f = np.zeros_like(X)
            for kk, a, p in zip(ks, amps, ph):
                f += a * np.sin(2 * math.pi * (kk[0] * X + kk[1] * Y + kk[2] * Z / 0.5) + p)
            W[v] = base[v] + f
        s.U[leaf] = boundary.prims_to_cons(W, 1.5)


def _divb_max(s):
    G = s.ghosted(s.U, s.t)
    return max(np.abs(_clib.divb(s.patch(b), G[b])).max() for b in s.forest.leaves)


@pytest.mark.parametrize("cd", [0.2, 0.8])
def test_periodic_box_of_blocks(cd):
    ic = _ic()
    g = _box()
    ora = solver.Solver(g, initial="zero", divb_cd=cd)
    _noisy_field(ora, 400)
    gpu = ic.Sim(g, divb_cd=cd)
    gpu.set_state(*ora.state(), 0.0)
    d0 = _divb_max(ora)
    for n in range(8):
        info = gpu.step()
        dt = ora.step()
        assert abs(info["dt_s"] / units.T0 - dt) <= 1e-12 * dt
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-12 * (n + 1), (n, e)
    assert _divb_max(ora) < d0


def test_refined_box_no_gradient_across_the_level_change():
    ic = _ic()
    g = _box(levels=2)
    ora = solver.Solver(g, initial="zero", divb_cd=0.5)
    _noisy_field(ora, 500)
    ora.regrid({b: (fo.REFINE if b in {(1, 0, 0, 0), (1, 1, 1, 0)} else fo.KEEP) for b in ora.forest.leaves},
               buffer_blocks=0)
    gpu = ic.Sim(g, amr=dict(buffer_blocks=0), divb_cd=0.5)
    gpu.set_state(*ora.state(), 0.0)
    for n in range(5):
        ora.step(1e-3)
        gpu.step(1e-3 * units.T0)
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-12 * (n + 1), (n, e)


@pytest.mark.parametrize("sch", ["two_stage", "hancock"])
def test_cme_wedge_with_cleaning(sch):
    ic = _ic()
    g, wind, cme, amr = tiny_wedge()
    ora = solver.Solver(g, wind, cme, amr, divb_cd=0.3, scheme=sch)
    gpu = ic.Sim(g, wind, [cme], amr, divb_cd=0.3, scheme=sch)
    gpu.set_state(*ora.state(), 0.0)
    for n in range(20):
        info = gpu.step()
        dt = ora.step()
        assert abs(info["dt_s"] / units.T0 - dt) <= 1e-12 * dt
        if n == 0:
            assert rel_err(gpu.state()[1], ora.state()[1]) <= 1e-12
    e = rel_err(gpu.state()[1], ora.state()[1])
    assert e <= 1e-10, e


def test_cleaning_coefficient_checked():
    ic = _ic()
    with pytest.raises(ic.ICError) as ex:
        ic.Sim(_box(), divb_cd=1.5)
    assert ex.value.status == ic.IC_E_INVALID
