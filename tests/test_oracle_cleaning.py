"""Pins of the oracle's parabolic div B cleaning (paper Sect. 2.1: parabolic
cleaning keeps div B errors small in every run).

The cleaning step moves B by dB = alpha C_d h^2 grad(div B) (h^2 = 1 / sum_d
dx_d^-2) and E by B . dB.  On a single Fourier mode B_x = eps sin(k x) of a
periodic box, the face-mean divergence and the central gradient give the
exact discrete decay factor 1 - alpha C_d (h^2 / dx^2) sin^2(k dx) per
application; repeated applications follow the diffusion equation
dB/dt = eta grad(div B), i.e. decay as exp(-n alpha C_d h^2 k^2), to
O((k dx)^2).  Total B is conserved on a periodic box (the gradient
telescopes), a uniform field is left alone, and cells on a non-periodic
boundary face get no normal gradient.
"""
import math

import numpy as np
import pytest

from oracle import _clib, boundary, geometry, solver

GAMMA = 1.5


def _box(n, L=(1.0, 0.5, 0.25), periodic=(True, True, True)):
    return dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=L, n=n, block=n, periodic=periodic,
                gamma=GAMMA, cfl=0.4)


def _mode_state(s, eps, m, L=1.0):
    nk, nj, ni = s.U.shape[1:]
    x = (np.arange(ni) + 0.5) * L / ni
    W = np.zeros((8, nk, nj, ni))
    W[0] = 1.0
    W[4] = 1.0
    W[5] = 0.3 + eps * np.sin(2 * math.pi * m * x / L)
    W[6] = -0.2
    W[7] = 0.4
    s.U = boundary.prims_to_cons(W, GAMMA)
    return x


def test_divb_closed_forms():
    # linear B_x = a x: the central form gives D = a exactly inside
    s = solver.PatchSolver(_box((8, 4, 4), periodic=(False, False, False)), initial="zero")
    G = np.zeros((8, 8, 8, 12))
    x = geometry.centres(s.geo.f[0])
    G[0] = 1.0
    G[4] = 1.0
    G[5] = 2.5 * x[None, None, :]
    G[6] = 0.7
    D = _clib.divb(s.pg, G)
    assert np.allclose(D, 2.5, rtol=1e-13, atol=0.0)
    G[5] = 0.3
    assert np.all(_clib.divb(s.pg, G) == 0.0)


@pytest.mark.parametrize("cd,alpha,m", [(0.2, 1.0, 1), (0.5, 0.5, 3), (0.9, 1.0, 5)])
def test_single_mode_exact_decay_factor(cd, alpha, m):
    n = (32, 4, 4)
    s = solver.PatchSolver(_box(n), initial="zero", divb_cd=cd)
    eps = 1e-3
    x = _mode_state(s, eps, m)
    U0 = s.U.copy()
    U1 = U0.copy()
    s.clean(U1, U0, 0.0, alpha)
    dx, dy, dz = 1.0 / 32, 0.5 / 4, 0.25 / 4
    h2 = 1.0 / (dx ** -2 + dy ** -2 + dz ** -2)
    k = 2 * math.pi * m
    fac = 1.0 - alpha * cd * (h2 / dx ** 2) * math.sin(k * dx) ** 2
    want = 0.3 + eps * fac * np.sin(k * x)
    assert np.allclose(U1[5], want[None, None, :], rtol=0.0, atol=1e-15)
    assert np.all(U1[6] == U0[6]) and np.all(U1[7] == U0[7])
    # energy moves by B . dB
    assert np.allclose(U1[4] - U0[4], U0[5] * (U1[5] - U0[5]), rtol=0.0, atol=1e-14)   # E is O(1)
    # total B_x is conserved on the periodic box
    assert abs(U1[5].sum() - U0[5].sum()) <= 1e-14 * abs(U0[5]).sum()


def test_repeated_cleaning_follows_the_diffusion_rate():
    """n applications decay the mode as (1 - c)^n with c -> alpha C_d h^2 k^2:
    the gap to exp(-n alpha C_d h^2 k^2) shrinks ~4x per grid doubling."""
    gaps = []
    for N in (16, 32, 64):
        s = solver.PatchSolver(_box((N, 4, 4), L=(1.0, 4.0 / N, 4.0 / N)), initial="zero", divb_cd=0.4)   # cubic cells
        eps = 1e-3
        _mode_state(s, eps, 1)
        dx = 1.0 / N
        h2 = 1.0 / (3 * dx ** -2)
        steps = int(round(0.02 / (0.4 * h2)))         # fixed diffusion "time" n C_d h^2
        U = s.U.copy()
        for _ in range(steps):
            V = U.copy()
            s.clean(V, U, 0.0, 1.0)
            U = V
        x = (np.arange(N) + 0.5) / N
        amp = 2.0 * np.mean((U[5, 0, 0] - 0.3) * np.sin(2 * math.pi * x))
        cont = eps * math.exp(-steps * 0.4 * h2 * (2 * math.pi) ** 2)
        gaps.append(abs(amp - cont) / cont)
    assert gaps[0] / gaps[1] > 3.0 and gaps[1] / gaps[2] > 3.0, gaps


def test_boundary_faces_get_no_normal_gradient():
    n = (16, 4, 4)
    s = solver.PatchSolver(_box(n, periodic=(False, True, True)), initial="zero", divb_cd=0.5)
    _mode_state(s, 1e-3, 1)
    U0 = s.U.copy()
    U1 = U0.copy()
    s.clean(U1, U0, 0.0, 1.0)
    assert np.all(U1[5, :, :, 0] == U0[5, :, :, 0]) and np.all(U1[5, :, :, -1] == U0[5, :, :, -1])
    assert np.any(U1[5, :, :, 5] != U0[5, :, :, 5])


def test_cleaning_damps_div_b_in_the_full_scheme():
    """At rest with uniform p and a div B error mode: with cleaning max|div B|
    falls well below the run without it (same steps)."""
    out = []
    for cd in (0.0, 0.5):
        s = solver.PatchSolver(_box((32, 4, 4)), initial="zero", divb_cd=cd)
        _mode_state(s, 1e-2, 2)
        for _ in range(40):
            s.step()
        G = s.ghosted(s.U, s.t)
        out.append(np.abs(_clib.divb(s.pg, G)).max())
    assert out[1] < 0.5 * out[0], out


def test_forest_cleaning_matches_the_patch_on_one_level():
    """The forest form (D across same-level block faces) equals the single
    patch form on a periodic box split into blocks."""
    n = (16, 8, 8)
    g = dict(_box(n, L=(1.0, 0.5, 0.5)), block=(8, 4, 4), max_level=1)
    p = solver.PatchSolver(dict(g, block=n), initial="zero", divb_cd=0.3)
    rng = np.random.default_rng(3)
    W = np.zeros((8,) + p.U.shape[1:])
    W[0] = 1.0
    W[4] = 1.0
    W[5:8] = rng.normal(0.0, 0.1, (3,) + p.U.shape[1:])
    p.U = boundary.prims_to_cons(W, GAMMA)
    f = solver.Solver(g, initial="zero", divb_cd=0.3)
    for leaf in f.forest.leaves:
        sl = tuple(slice(leaf[1 + d] * g["block"][d], (leaf[1 + d] + 1) * g["block"][d]) for d in (2, 1, 0))
        f.U[leaf] = p.U[(slice(None),) + sl].copy()
    U1 = p.U.copy()
    p.clean(U1, p.U, 0.0, 1.0)
    G = f.ghosted(f.U, 0.0)
    V = {b: u.copy() for b, u in f.U.items()}
    f.clean(V, G, 1.0)
    for leaf in f.forest.leaves:
        sl = tuple(slice(leaf[1 + d] * g["block"][d], (leaf[1 + d] + 1) * g["block"][d]) for d in (2, 1, 0))
        assert np.allclose(V[leaf], U1[(slice(None),) + sl], rtol=1e-15, atol=1e-17)
