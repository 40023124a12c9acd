"""Pins of the oracle's block-AMR machinery.

- restriction of a prolongation is the identity, and a linear field is
  prolonged exactly where the limiter is inactive (conservative, centroid
  based prolongation); where linear values would make a child's pressure
  negative (a cold linear velocity ramp, closed form below) the children
  take the parent's value;
- one-level forests give the same state, bit for bit, as the single-patch
  solver (the block decomposition and ghost exchange change nothing);
- a two-level periodic box with reflux conserves sum(V U) to round-off, and a
  uniform state at rest on a two-level stretched wedge stays uniform;
- the regrid logic against a brute-force fixpoint on small forests, and the
  forest invariants (2:1 over 26 neighbours, nesting, covered volume).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import boundary, forest as fo, solver
from synthetic import smooth_modes, workload, as_dict


def _box(levels=2, n=(16, 8, 8), block=(4, 4, 4), periodic=(True, True, True)):
    return dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 0.5, 0.5), n=n, block=block,
                periodic=periodic, max_level=levels, gamma=1.5, cfl=0.4)


def _smooth_state(s, seed=100):
    for leaf in s.forest.leaves:
        g = s.geo[leaf[0]]
        x = [np.array([g.centre(d, m) for m in range(*s.cell_range(leaf, d))]) for d in range(3)]
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        W = np.zeros((8,) + X.shape)
        base = [1.0, 0.0, 0.0, 0.0, 1.0, 0.3, 0.2, -0.1]
        for v in range(8):
            ks, amps, ph = smooth_modes(seed + v, 3, 0.2 if v in (0, 4) else 0.3)
            f = np.zeros_like(X)
            for kk, a, p in zip(ks, amps, ph):
                f += a * np.sin(2 * math.pi * (kk[0] * X + 2 * kk[1] * Y + 2 * kk[2] * Z) + p)
            W[v] = base[v] + f
        s.U[leaf] = boundary.prims_to_cons(W, s.gamma)


def _refine(s, leaves):
    flags = {b: (fo.REFINE if b in leaves else fo.KEEP) for b in s.forest.leaves}
    s.regrid(flags, buffer_blocks=0)


def test_restrict_of_prolong_is_identity():
    s = solver.Solver(_box(), initial="zero")
    _smooth_state(s)
    parent = (1, 1, 0, 1)
    U0 = s.U[parent].copy()
    _refine(s, {parent})
    gidx = [np.arange(parent[1 + d] * 4, (parent[1 + d] + 1) * 4) for d in range(3)]
    back = s.restrict(s.U, 1, gidx)
    assert np.allclose(back, U0, rtol=1e-14, atol=1e-14)


def test_linear_field_prolonged_exactly():
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 60.0), n=(16, 8, 16),
                block=(8, 4, 4), stretched_r=True, max_level=2, gamma=1.5,
                bc=[("outflow", "outflow")] * 3)
    s = solver.Solver(grid, initial="zero")
    parent = (1, 1, 1, 1)
    # a field linear in (r, theta, phi) in every variable: the minmod slopes equal
    # the gradient, and the centroid-based prolongation reproduces the child's
    # volume average exactly only along phi; along r and theta it reproduces
    # the linear function at the child's centroid
    g1, g2 = s.geo[1], s.geo[2]
    for leaf in s.forest.leaves:
        x = [np.array([g1.centre(d, m) for m in range(*s.cell_range(leaf, d))]) for d in range(3)]
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        # physical everywhere (energy offset large), so no positivity fallback
        s.U[leaf] = np.stack([1.0 + 0.5 * X + 0.3 * Y + 0.2 * Z + (40.0 if v == 4 else 0.1 * v) for v in range(8)])
    G = s.ghosted(s.U, 0.0)
    ch = (2, 2, 2, 2)   # its parent cells and their neighbours are away from the boundary
    gidx = [np.arange(ch[1 + d] * np.array(grid["block"])[d], (ch[1 + d] + 1) * grid["block"][d]) for d in range(3)]
    val = s.prolong(G[parent], parent, 2, gidx)
    for c, (k, j, i) in enumerate(itertools.product(range(4), range(4), range(8))):
        gi, gj, gk = gidx[0][i], gidx[1][j], gidx[2][k]
        # linear function at the child's centre, shifted by the parent's offset
        # between its own centre and its children's volume centroid
        pc = [gi // 2, gj // 2, gk // 2]
        xbar = []
        for d, (a, pidx) in enumerate(zip((gi, gj, gk), pc)):
            c0, c1 = 2 * pidx, 2 * pidx + 1
            w0, w1 = g2.volume_weight(d, c0), g2.volume_weight(d, c1)
            xbar.append((w0 * g2.centre(d, c0) + w1 * g2.centre(d, c1)) / (w0 + w1))
        xf = [g2.centre(0, gi), g2.centre(1, gj), g2.centre(2, gk)]
        xc = [g1.centre(0, pc[0]), g1.centre(1, pc[1]), g1.centre(2, pc[2])]
        lin = lambda x: 1.0 + 0.5 * x[0] + 0.3 * x[1] + 0.2 * x[2]
        expect = lin(xc) + 0.5 * (xf[0] - xbar[0]) + 0.3 * (xf[1] - xbar[1]) + 0.2 * (xf[2] - xbar[2])
        assert abs(val[0, k, j, i] - expect) < 1e-13
    del c


def test_prolongation_is_conservative():
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 60.0), n=(16, 8, 8),
                block=(8, 4, 4), stretched_r=True, max_level=2, gamma=1.5,
                bc=[("outflow", "outflow")] * 3)
    s = solver.Solver(grid, initial="zero")
    rng = np.random.default_rng(3)
    for leaf in s.forest.leaves:
        s.U[leaf] = 1.0 + rng.uniform(0, 1, s.U[leaf].shape)
    tot0 = s.total()
    _refine(s, {(1, 0, 1, 1), (1, 1, 0, 0)})
    assert np.allclose(s.total(), tot0, rtol=1e-14)


@pytest.mark.parametrize("P", [0.05, 0.5])
def test_prolongation_positivity_fallback(P):
    """rho = 1, v_x = k x, B = 0, p/(gamma-1) = P on a uniform Cartesian grid
    of spacing h.  m_x is linear and prolonged exactly; E = k^2 x^2 / 2 + P has
    the one-sided slopes k^2 (x -+ h/2), minmod takes the smaller one, and the
    children of cell x > 0 get p/(gamma-1) = P + 3 k^2 h^2 / 32 at x - h/4 and
    P - 5 k^2 h^2 / 32 at x + h/4.  With k h = 1 the latter is negative for
    P = 0.05, so every child takes its parent's value; for P = 0.5 both are
    positive and the linear values stay."""
    g = _box(levels=2, n=(16, 4, 4), block=(4, 4, 4), periodic=(False, True, True))
    g["x1"] = (16.0, 4.0, 4.0)             # h = 1
    s = solver.Solver(g, initial="zero")
    k = 1.0
    for leaf in s.forest.leaves:
        x = np.array([s.geo[1].centre(0, m) for m in range(*s.cell_range(leaf, 0))])
        U = np.zeros((8, 4, 4, 4))
        U[0] = 1.0
        U[1] = k * x[None, None, :]
        U[4] = 0.5 * (k * x[None, None, :]) ** 2 + P
        s.U[leaf] = U
    parent = (1, 2, 0, 0)                  # cells x = 8.5 .. 11.5, interior
    U0 = s.U[parent].copy()
    tot0 = s.total()
    _refine(s, {parent})
    kids = [b for b in s.forest.leaves if b[0] == 2]
    assert len(kids) == 8
    for ch in kids:
        Uf = s.U[ch]
        for i in range(4):
            gi = ch[1] * 4 + i                 # fine global index, fine spacing h / 2
            pc = gi // 2 - 8                   # parent-local cell
            if P == 0.05:
                assert np.array_equal(Uf[:, :, :, i], np.broadcast_to(U0[:, :, :, pc], Uf[:, :, :, i].shape))
            else:
                assert np.allclose(Uf[1, :, :, i], k * (gi + 0.5) * 0.5, rtol=1e-14)
                eint = Uf[4, :, :, i] - 0.5 * Uf[1, :, :, i] ** 2 / Uf[0, :, :, i]
                expect = P + (3.0 if gi % 2 == 0 else -5.0) * k ** 2 / 32.0
                assert np.allclose(eint, expect, rtol=1e-12)
    assert np.allclose(s.total(), tot0, rtol=1e-14)


def test_single_level_blocks_equal_single_patch():
    w = workload("tiny_wedge")
    g, wind, cme = as_dict(w.grid), as_dict(w.wind), as_dict(w.cmes[0])
    a = solver.Solver(g, wind, cme, as_dict(w.amr))
    b = solver.PatchSolver(g, wind, cme)
    for _ in range(4):
        assert a.step() == b.step()
    bl, U = a.state()
    bl2, U2 = b.to_blocks(g["block"])
    assert bl == bl2 and np.array_equal(U, U2)


def test_two_level_periodic_box_conserves():
    s = solver.Solver(_box(), initial="zero")
    _smooth_state(s)
    _refine(s, {(1, 1, 0, 1), (1, 2, 1, 1), (1, 1, 1, 1)})
    assert any(b[0] == 2 for b in s.forest.leaves)
    tot0 = s.total()
    scale = np.zeros(8)
    for leaf, u in s.U.items():
        scale += np.abs(u).reshape(8, -1).sum(axis=1)
    scale *= (1.0 / 16) * (0.5 / 8) * (0.5 / 8) / 8
    for _ in range(20):
        s.step()
    assert np.all(np.abs(s.total() - tot0) <= 1e-13 * scale * 8), (s.total() - tot0) / scale


def test_two_level_wedge_free_stream():
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 60.0), n=(16, 8, 8),
                block=(4, 4, 4), stretched_r=True, max_level=2, gamma=1.5, cfl=0.4,
                bc=[("outflow", "outflow")] * 3)
    s = solver.Solver(grid, omega=0.0, gm=0.0, initial="zero")
    W = np.zeros((8, 4, 4, 4))
    W[0], W[4] = 2.0, 0.7
    for leaf in s.forest.leaves:
        s.U[leaf] = boundary.prims_to_cons(W, 1.5)
    _refine(s, {(1, 1, 0, 1), (1, 2, 1, 0)})
    for _ in range(20):
        s.step()
    dev = max(np.abs(u - boundary.prims_to_cons(W, 1.5)).max() for u in s.U.values())
    assert dev <= 1e-13, dev


# --- forest ---------------------------------------------------------------------

def _brute_regrid(F, flags, buffer_blocks):
    """Regrid by brute force over all leaf pairs."""
    leaves = sorted(F.leaves)
    f = {b: flags.get(b, fo.KEEP) for b in leaves}
    for b in leaves:
        if f[b] == fo.REFINE and b[0] >= F.max_level:
            f[b] = fo.KEEP
        if f[b] == fo.COARSEN and b[0] <= 1:
            f[b] = fo.KEEP

    def face_touch(a, b):
        # share a face of positive area: touch in 3 dims, overlap with positive
        # length in exactly 2 of them
        L = max(a[0], b[0], F.max_level)
        ea, eb = F.extent(a, L), F.extent(b, L)
        n = F.nblocks(L)
        if not F.touch(a, b):
            return False
        pos = 0
        for d in range(3):
            shifts = (-n[d], 0, n[d]) if F.periodic[d] else (0,)
            if any(min(ea[d][1], eb[d][1] + s) - max(ea[d][0], eb[d][0] + s) > 0 for s in shifts):
                pos += 1
        return pos == 2

    orig = [b for b in leaves if f[b] == fo.REFINE]
    for b in orig:
        for n in leaves:
            if n != b and face_touch(b, n):
                if buffer_blocks and n[0] < F.max_level and n[0] <= b[0]:
                    f[n] = fo.REFINE
                elif f[n] == fo.COARSEN:
                    f[n] = fo.KEEP
    changed = True
    while changed:
        changed = False
        for a in leaves:
            for b in leaves:
                if f[a] == fo.REFINE and b[0] == a[0] - 1 and f[b] != fo.REFINE and F.touch(a, b):
                    f[b] = fo.REFINE
                    changed = True
    post = set()
    for b in leaves:
        if f[b] == fo.REFINE:
            for o in range(8):
                post.add((b[0] + 1, 2 * b[1] + (o & 1), 2 * b[2] + ((o >> 1) & 1), 2 * b[3] + ((o >> 2) & 1)))
        else:
            post.add(b)
    groups = {}
    for b in leaves:
        if f[b] == fo.COARSEN:
            groups.setdefault((b[0] - 1, b[1] // 2, b[2] // 2, b[3] // 2), []).append(b)
    new = set(post)
    for p, ch in groups.items():
        if len(ch) < 8:
            continue
        if any(q[0] >= p[0] + 2 and F.touch(p, q) for q in post):
            continue
        for c in ch:
            new.discard(c)
        new.add(p)
    return new


def _random_forest(rng, nb, periodic, max_level, steps=3):
    F = fo.Forest(nb, periodic, max_level)
    for _ in range(steps):
        flags = {b: int(rng.choice([fo.REFINE, fo.KEEP, fo.COARSEN], p=[0.25, 0.5, 0.25])) for b in F.leaves}
        new, _, _ = F.regrid(flags, 0)
        F = fo.Forest(nb, periodic, max_level, new)
    return F


@pytest.mark.parametrize("seed", range(12))
def test_regrid_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    nb = tuple(int(x) for x in rng.integers(1, 4, size=3))
    periodic = tuple(bool(x) for x in rng.integers(0, 2, size=3))
    F = _random_forest(rng, nb, periodic, 3)
    for buffer_blocks in (0, 1):
        flags = {b: int(rng.choice([fo.REFINE, fo.KEEP, fo.COARSEN], p=[0.2, 0.3, 0.5])) for b in F.leaves}
        new, _, _ = F.regrid(flags, buffer_blocks)
        assert new == _brute_regrid(F, flags, buffer_blocks)
        G = fo.Forest(nb, periodic, 3, new)
        assert G.check_balance()
        # the leaves tile the domain: total volume in finest-block units
        vol = sum(8 ** (3 - b[0]) for b in new)
        assert vol == nb[0] * nb[1] * nb[2] * 8 ** 2


def test_morton_order_interleaves_bits():
    assert fo.morton(1, 0, 0) == 1 and fo.morton(0, 1, 0) == 2 and fo.morton(0, 0, 1) == 4
    assert fo.morton(3, 0, 0) == 9 and fo.morton(2, 2, 2) == 56
