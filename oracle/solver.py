"""Oracle solvers: one ghosted patch, or a block-AMR forest (test infrastructure only).

Time step (paper Sect. 2.1, second order in time; two-stage midpoint form):
    stage 1: ghosts at t^n,        U*      = U^n + (dt/2) L(U^n)
    stage 2: ghosts at t^n + dt/2, U^{n+1} = U^n +  dt    L(U*)
    dt = C_cfl / max_cells sum_d (|v_d| + c_f,d) / dx_d, computed on U^n.
Scheme variants (Sect. 2.1 names further scheme and limiter combinations):
the limiter of the reconstruction (monotonised central, minmod, van Leer),
and the Hancock one-step form, whose first stage is the predictor
U* = U^n + (dt/2) L_H(U^n) (each cell's own physical fluxes at its
reconstructed face states; no interface solver, no reflux), followed by the
same second stage.

Parabolic div B cleaning (Sect. 2.1 applies it in every run; off by default
here): after each stage's update (reflux and floors included) the field of
the stage result moves by dB = alpha C_d h^2 grad(D), D the discrete div B of
the stage input (face-mean form), grad(D) by central differences of D between
the face neighbours in physical components, h^2 = 1 / sum_d dx_d^-2 with the
cell widths of the CFL rate, alpha the stage weight (1/2, 1); the energy
moves by B_in . dB.  A gradient component that would need D across a
physical boundary or a level change is zero (the cleaning stays out of the
cells on those faces).

Density tracer (Sect. 3.1, an option): a ninth conserved variable rho s, s the
CME mass fraction (1 in the cone CME injected at the inner boundary, 0 in the
wind and initially), advected by the same TVDLF flux, no source; floors
leave it.  Refinement criteria (amr "criterion"): "shock" (the Sect. 3.2
criterion), "tracer" (Sect. 3.1: refine where the tracer is present, s >
tracer_refine in some cell; coarsen where s <= tracer_coarsen everywhere; no
windows) and "combined" (Sect. 3.3: inside the windows, the shock condition
or the tracer condition).

Block AMR (Sect. 3): every leaf carries two face-ghost layers per face.  Face
ghosts come from a same-level neighbour (copy), from finer neighbours
(volume-weighted restriction of the 8 children of each ghost cell) or from a
coarser neighbour (conservative, minmod-limited linear prolongation around the
children's volume centroid); coarse ghosts are filled before fine ones, so a
prolongation can use the coarse block's own ghosts.  At coarse-fine faces
the coarse cell's flux is replaced by the area-weighted sum of the four fine
face fluxes in every stage (reflux), which keeps sum(V U) conserved.
All leaves advance with one global dt (no subcycling).
"""
import math

import numpy as np

from . import _clib, boundary, forest as fo, geometry, units

NV = 8


def _bc_of(grid):
    if grid.get("bc") is not None:
        return [tuple(x) for x in grid["bc"]]
    per = grid.get("periodic", (False, False, False))
    if grid["geometry"] == "cartesian":
        return [("periodic", "periodic") if per[d] else ("outflow", "outflow") for d in range(3)]
    return [("inner", "outflow"), ("outflow", "outflow"),
            ("periodic", "periodic") if per[2] else ("outflow", "outflow")]


def _phys(grid, omega, gm):
    cart = grid["geometry"] == "cartesian"
    om = 0.0 if cart else (units.OMEGA_CODE if omega is None else omega)
    g = 0.0 if cart else (units.GM_CODE if gm is None else gm)
    return om, g


class UnphysicalState(RuntimeError):
    pass


# Small-value floors (code units), applied to every stage result: a cell with
# rho < RHO_FLOOR takes rho = RHO_FLOOR at zero velocity (m / rho of a
# collapsing density is meaningless, and keeping it plants runaway speeds);
# then a cell with p < P_FLOOR has its energy raised so that p = P_FLOOR.  The paper's scheme is
# not positivity preserving and it does not say how its code treats small
# values; a fast CME followed by slow wind opens a near-vacuum rarefaction
# behind the CME, where the exact update undershoots to p < 0.
RHO_FLOOR = 1.0e-6
P_FLOOR = 1.0e-9


def apply_floors(U, gamma, rho_floor=RHO_FLOOR, p_floor=P_FLOOR, counts=None):
    """Floors on a conserved array [8, ...] (in place); returns the number of
    floor actions (density-floored cells plus pressure-floored cells).  counts,
    if a list [n_rho, n_p], has the two numbers added to it."""
    n = 0
    low = U[0] < rho_floor
    n_rho = int(low.sum())
    if n_rho:
        U[1:4] = np.where(low, 0.0, U[1:4])
        U[0] = np.where(low, rho_floor, U[0])
        n += n_rho
    kin = 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]
    mag = 0.5 * (U[5] ** 2 + U[6] ** 2 + U[7] ** 2)
    p = (gamma - 1.0) * (U[4] - kin - mag)
    lowp = p < p_floor
    n_p = int(lowp.sum())
    if n_p:
        U[4] = np.where(lowp, p_floor / (gamma - 1.0) + kin + mag, U[4])
        n += n_p
    if counts is not None:
        counts[0] += n_rho
        counts[1] += n_p
    return n


def _cleaning_metric(cart, c, w, sp):
    """(dx, gs): per direction, the cell widths of the CFL rate (dr, r_c dtheta,
    r_c sin(theta_c) dphi) and the spacings of the central gradient in physical
    components (x_{m+1} - x_{m-1}, times r_c and r_c sin(theta_c)), shaped to
    broadcast over [k, j, i].  c: centres of cells -1 .. n, w: widths of cells
    0 .. n-1, sp: centre spacings per direction."""
    shape = lambda a, d: a.reshape([-1 if e == 2 - d else 1 for e in range(3)])
    if cart:
        return [shape(w[d], d) for d in range(3)], [shape(sp[d], d) for d in range(3)]
    rc, tc = shape(c[0][1:-1], 0), shape(c[1][1:-1], 1)
    dx = [shape(w[0], 0), rc * shape(w[1], 1), rc * np.sin(tc) * shape(w[2], 2)]
    gs = [shape(sp[0], 0), rc * shape(sp[1], 1), rc * np.sin(tc) * shape(sp[2], 2)]
    return dx, gs


def _apply_cleaning(u, G, Dp, dx, gs, coef):
    """u += the cleaning increment: dB_d = coef h^2 (D_{+d} - D_{-d}) / gs_d (0
    where a neighbour's D is missing, NaN in Dp), E += B_in . dB."""
    h2 = 1.0 / (1.0 / dx[0] ** 2 + 1.0 / dx[1] ** 2 + 1.0 / dx[2] ** 2)
    Bin = G[5:8, 2:-2, 2:-2, 2:-2]
    for d in range(3):
        ax = 2 - d
        hi, lo = [slice(1, -1)] * 3, [slice(1, -1)] * 3
        hi[ax], lo[ax] = slice(2, None), slice(0, -2)
        grad = (Dp[tuple(hi)] - Dp[tuple(lo)]) / gs[d]
        dB = coef * h2 * np.where(np.isnan(grad), 0.0, grad)
        u[4] += Bin[d] * dB
        u[5 + d] += dB


# refinement-criterion readings: Loehner eps, thresholds, weights, the
# Earth/CME windows of Sect. 3.2, regrid cadence and buffer
AMR_DEFAULTS = dict(eps_lohner=0.01, tol_refine=0.1, tol_coarsen=0.0125, w_rho=0.5, w_v=0.5,
                    lon_earth_deg=0.0, clt_earth_deg=90.0, dlon_earth_deg=30.0,
                    dclt_earth_deg=10.0, dlon_cme_deg=90.0, use_windows=True,
                    regrid_every=10, buffer_blocks=1, criterion="shock",
                    tracer_refine=0.01, tracer_coarsen=0.00125)


class Solver:
    """Block-forest solver.  State: dict leaf -> U[8, bk, bj, bi] (code units)."""

    def __init__(self, grid, wind=None, cme=None, amr=None, omega=None, gm=None, t0_s=0.0,
                 initial="wind", rho_floor=RHO_FLOOR, p_floor=P_FLOOR, limiter="mc", scheme="two_stage",
                 divb_cd=0.0, tracer=False):
        self.rho_floor, self.p_floor, self.floored = rho_floor, p_floor, 0
        self.limiter, self.scheme, self.divb_cd = limiter, scheme, float(divb_cd)
        self.nv = 9 if tracer else NV
        assert scheme in ("two_stage", "hancock")
        self.floor_counts = [0, 0]         # density-floored, pressure-floored cells
        self.grid = dict(grid)
        self.grid.setdefault("geometry", "spherical")
        self.grid.setdefault("periodic", (False, False, False))
        self.grid.setdefault("stretched_r", False)
        self.grid.setdefault("max_level", 1)
        self.cart = self.grid["geometry"] == "cartesian"
        self.B = tuple(int(b) for b in self.grid["block"])
        n = self.grid["n"]
        for d in range(3):
            if n[d] % self.B[d]:
                raise ValueError("cells per direction must be a multiple of the block size")
        self.nb = tuple(n[d] // self.B[d] for d in range(3))
        self.gamma = float(self.grid.get("gamma", 1.5))
        self.cfl = float(self.grid.get("cfl", 0.4))
        self.omega, self.gm = _phys(self.grid, omega, gm)
        self.bc = _bc_of(self.grid)
        self.wind = wind
        self.cme = cme
        self.amr = dict(AMR_DEFAULTS)
        self.amr.update(amr or {})
        self.max_level = int(self.grid["max_level"])
        self.geo = [None] + [geometry.LevelGeometry(self.grid, l) for l in range(1, self.max_level + 2)]
        self.r_in = self.geo[1].f[0][2]
        self.forest = fo.Forest(self.nb, self.grid["periodic"], self.max_level)
        self.t = units.time_code(t0_s)
        self.steps = 0
        self._patch = {}
        self.U = {}
        if initial == "wind" and wind is not None and not self.cart:
            for b in self.forest.leaves:
                self.U[b] = self.initial_block(b)
        else:
            for b in self.forest.leaves:
                self.U[b] = np.zeros((self.nv,) + self.B[::-1])

    # --- geometry -------------------------------------------------------------
    def cell_range(self, leaf, d):
        lo = leaf[1 + d] * self.B[d]
        return lo, lo + self.B[d]

    def patch(self, leaf):
        if leaf not in self._patch:
            g = self.geo[leaf[0]]
            f = [g.faces(d, *self.cell_range(leaf, d)) for d in range(3)]
            self._patch[leaf] = _clib.PatchGeom(f[0], f[1], f[2], self.cart, self.gamma,
                                                self.omega, self.gm, self.limiter, self.nv)
        return self._patch[leaf]

    def centres(self, leaf, d, lo=0, hi=None):
        g = self.geo[leaf[0]]
        a, _ = self.cell_range(leaf, d)
        hi = self.B[d] if hi is None else hi
        return np.array([g.centre(d, a + m) for m in range(lo, hi)])

    def initial_block(self, leaf):
        r = self.centres(leaf, 0)[None, None, :]
        th = self.centres(leaf, 1)[None, :, None]
        ph = self.centres(leaf, 2)[:, None, None]
        W = boundary.initial_prims(self.wind, r, th, ph, self.r_in, self.omega, self.gamma)
        if self.nv > NV:
            W = np.concatenate([W, np.zeros((1,) + W.shape[1:])])      # no CME material yet
        return boundary.prims_to_cons(W, self.gamma)

    # --- ghost cells ----------------------------------------------------------
    @staticmethod
    def _slab(d, side, B):
        """Index expression of the two ghost layers of face (d, side) in a
        ghosted array [v, k, j, i]."""
        sl = [slice(None), slice(2, 2 + B[2]), slice(2, 2 + B[1]), slice(2, 2 + B[0])]
        ax = 3 - d
        sl[ax] = slice(0, 2) if side == 0 else slice(2 + B[d], 4 + B[d])
        return tuple(sl)

    def _slab_global(self, leaf, d, side):
        """Global (level, unwrapped) cell indices of the ghost slab, per direction."""
        out = []
        for e in range(3):
            lo, hi = self.cell_range(leaf, e)
            if e == d:
                out.append(np.arange(lo - 2, lo) if side == 0 else np.arange(hi, hi + 2))
            else:
                out.append(np.arange(lo, hi))
        return out

    def ghosted(self, U, t):
        """Ghosted arrays of all leaves for state U at code time t."""
        G = {}
        for leaf in sorted(self.forest.leaves):  # ascending level
            g = np.zeros((self.nv,) + tuple(b + 4 for b in self.B[::-1]))
            g[:, 2:-2, 2:-2, 2:-2] = U[leaf]
            for d in range(3):
                for side in (0, 1):
                    self._fill_face(g, leaf, d, side, U, G, t)
            G[leaf] = g
        return G

    def _fill_face(self, g, leaf, d, side, U, G, t):
        B = self.B
        sl = self._slab(d, side, B)
        nbs = self.forest.face_neighbours(leaf, d, side)
        if not nbs:
            kind = self.bc[d][side]
            if kind == "outflow":
                src = [slice(None), slice(2, 2 + B[2]), slice(2, 2 + B[1]), slice(2, 2 + B[0])]
                ax = 3 - d
                edge = 2 if side == 0 else 1 + B[d]
                src[ax] = slice(edge, edge + 1)
                g[sl] = g[tuple(src)]
            elif kind == "inner":
                th = self.centres(leaf, 1)[None, :, None]
                ph = self.centres(leaf, 2)[:, None, None]
                W = boundary.boundary_prims(self.wind, self.cme, th + 0.0 * ph, ph + 0.0 * th,
                                            self.r_in, self.omega, t)
                if self.nv > NV:      # CME material: s = 1 inside the cone, 0 in the wind
                    s_in = boundary.cme_mask(self.cme, th + 0.0 * ph, ph + 0.0 * th, self.r_in, t) \
                        if self.cme is not None else np.zeros(W.shape[1:], dtype=bool)
                    W = np.concatenate([W, s_in[None].astype(np.float64)])
                g[sl] = boundary.prims_to_cons(W, self.gamma)    # [v, k, j, 1]
            else:
                raise ValueError("boundary kind %r without a neighbour" % kind)
            return
        nl = nbs[0][0]
        if nl == leaf[0]:
            src = U[nbs[0]]
            sel = [slice(None)] * 4
            ax = 3 - d
            sel[ax] = slice(B[d] - 2, B[d]) if side == 0 else slice(0, 2)
            g[sl] = src[tuple(sel)]
        elif nl < leaf[0]:
            gidx = self._slab_global(leaf, d, side)
            g[sl] = self.prolong(G[nbs[0]], nbs[0], leaf[0], gidx)
        else:
            gidx = self._slab_global(leaf, d, side)
            g[sl] = self.restrict(U, leaf[0], gidx)

    def _wrap_idx(self, level, d, idx):
        n = self.geo[level].n[d]
        return np.mod(idx, n) if self.grid["periodic"][d] else idx

    def _centroid_offsets(self, level_f, d, gf):
        """x_f - xbar of fine cells gf (level level_f) along d, where xbar is the
        volume centroid of the two children of their coarse parent along d."""
        g = self.geo[level_f]
        gc = gf // 2
        out = np.empty(len(gf))
        for n, (a, c) in enumerate(zip(gf, gc)):
            c0, c1 = 2 * c, 2 * c + 1
            w0, w1 = g.volume_weight(d, c0), g.volume_weight(d, c1)
            xbar = (w0 * g.centre(d, c0) + w1 * g.centre(d, c1)) / (w0 + w1)
            out[n] = g.centre(d, a) - xbar
        return out

    def prolong(self, Gc, cleaf, level_f, gidx):
        """Values of fine cells (global indices gidx per direction, level level_f)
        by limited linear prolongation from coarse leaf cleaf with ghosted array Gc."""
        gc_geo = self.geo[level_f - 1]
        loc, off, coarse_glob = [], [], []
        for d in range(3):
            gf = self._wrap_idx(level_f, d, np.asarray(gidx[d]))
            gcg = gf // 2
            lo, _ = self.cell_range(cleaf, d)
            loc.append(gcg - lo)
            coarse_glob.append(gcg)
            off.append(self._centroid_offsets(level_f, d, gf))
        K, J, I = np.meshgrid(loc[2], loc[1], loc[0], indexing="ij")
        Uc = Gc[:, K + 2, J + 2, I + 2]
        out = Uc.copy()
        slopes, sib = [], []
        for d in range(3):
            cg = coarse_glob[d]
            xm = np.array([gc_geo.centre(d, c - 1) for c in cg])
            x0 = np.array([gc_geo.centre(d, c) for c in cg])
            xp = np.array([gc_geo.centre(d, c + 1) for c in cg])
            shp = [1, 1, 1]
            shp[2 - d] = len(cg)
            step = [0, 0, 0]
            step[2 - d] = 1
            Um = Gc[:, K + 2 - step[0], J + 2 - step[1], I + 2 - step[2]]
            Up = Gc[:, K + 2 + step[0], J + 2 + step[1], I + 2 + step[2]]
            a = (Uc - Um) / (x0 - xm).reshape(shp)
            b = (Up - Uc) / (xp - x0).reshape(shp)
            s = np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)
            out = out + s * off[d].reshape(shp)
            slopes.append(s)
            gf = self._wrap_idx(level_f, d, np.asarray(gidx[d]))
            sib.append([self._centroid_offsets(level_f, d, 2 * (gf // 2) + o).reshape(shp) for o in (0, 1)])
        # positivity: a coarse cell whose linear values would give any of its 8
        # children rho <= 0 or p <= 0 passes its own value to all of them
        ok = np.ones(Uc.shape[1:], dtype=bool)
        for o in range(8):
            c = Uc + slopes[0] * sib[0][o & 1]
            c = c + slopes[1] * sib[1][(o >> 1) & 1]
            c = c + slopes[2] * sib[2][(o >> 2) & 1]
            with np.errstate(divide="ignore", invalid="ignore"):
                p = c[4] - 0.5 * (c[1] ** 2 + c[2] ** 2 + c[3] ** 2) / c[0] - 0.5 * (c[5] ** 2 + c[6] ** 2 + c[7] ** 2)
            ok &= (c[0] > 0.0) & (p > 0.0)
        return np.where(ok[None], out, Uc)

    def restrict(self, U, level_c, gidx):
        """Values of coarse cells (global indices gidx, level level_c) as the
        volume-weighted mean of their 8 children, read from the leaves of level_c+1."""
        gf_geo = self.geo[level_c + 1]
        gw = [self._wrap_idx(level_c, d, np.asarray(gidx[d])) for d in range(3)]
        shape = (self.nv, len(gw[2]), len(gw[1]), len(gw[0]))
        num = np.zeros(shape)
        den = np.zeros(shape[1:])
        for o in range(8):
            oz, oy, ox = (o >> 2) & 1, (o >> 1) & 1, o & 1
            fi, fj, fk = 2 * gw[0] + ox, 2 * gw[1] + oy, 2 * gw[2] + oz
            wi = np.array([gf_geo.volume_weight(0, x) for x in fi])
            wj = np.array([gf_geo.volume_weight(1, x) for x in fj])
            wk = np.array([gf_geo.volume_weight(2, x) for x in fk])
            w = wk[:, None, None] * wj[None, :, None] * wi[None, None, :]
            vals = np.empty(shape)
            for a, z in enumerate(fk):
                for bb, y in enumerate(fj):
                    for c, x in enumerate(fi):
                        lf = (level_c + 1, x // self.B[0], y // self.B[1], z // self.B[2])
                        arr = U[lf]
                        vals[:, a, bb, c] = arr[:, z - lf[3] * self.B[2], y - lf[2] * self.B[1],
                                                x - lf[1] * self.B[0]]
            num += w * vals
            den += w
        return num / den

    # --- spatial operator -----------------------------------------------------
    def metric(self, leaf, d, i, j, k):
        """(am, ap) = A_face/V of local cell (i, j, k) of `leaf` along d (same
        algebraic form as the C core)."""
        g = self.geo[leaf[0]]
        gi = i + self.cell_range(leaf, 0)[0]
        gj = j + self.cell_range(leaf, 1)[0]
        gk = k + self.cell_range(leaf, 2)[0]
        f = g.f
        if self.cart:
            m = (gi, gj, gk)[d]
            w = f[d][m + 3] - f[d][m + 2]
            return 1.0 / w, 1.0 / w
        rm, rp = f[0][gi + 2], f[0][gi + 3]
        tm, tp = f[1][gj + 2], f[1][gj + 3]
        dr3 = rp * rp * rp - rm * rm * rm
        rtinv = 1.5 * (rp * rp - rm * rm) / dr3
        dmu = math.cos(tm) - math.cos(tp)
        if d == 0:
            return 3.0 * rm * rm / dr3, 3.0 * rp * rp / dr3
        if d == 1:
            return rtinv * math.sin(tm) / dmu, rtinv * math.sin(tp) / dmu
        dphi = f[2][gk + 3] - f[2][gk + 2]
        a = rtinv * (tp - tm) / (dmu * dphi)
        return a, a

    def operator(self, U, t):
        """L(U) for every leaf, with reflux at coarse-fine faces."""
        G = self.ghosted(U, t)
        L, F = {}, {}
        bad = 0
        for leaf in self.forest.leaves:
            L[leaf], F[leaf], nb = _clib.rhs(self.patch(leaf), G[leaf])
            bad += nb
        if bad:
            raise UnphysicalState("%d cells with rho <= 0, p <= 0 or non-finite values" % bad)
        self._reflux(L, F)
        return L, G

    def predictor(self, U, t):
        """Hancock predictor operator L_H(U) of every leaf (ghosts at t)."""
        G = self.ghosted(U, t)
        L = {}
        bad = 0
        for leaf in self.forest.leaves:
            L[leaf], nb = _clib.rhs_hancock(self.patch(leaf), G[leaf])
            bad += nb
        if bad:
            raise UnphysicalState("%d cells with rho <= 0, p <= 0 or non-finite values" % bad)
        return L, G

    def _widths(self, leaf):
        """Per-direction arrays (broadcast over [k, j, i]) of the cell widths of
        the CFL rate and the central-difference spacings of the gradient."""
        g = self.geo[leaf[0]]
        rng = [self.cell_range(leaf, d) for d in range(3)]
        c = [np.array([g.centre(d, m) for m in range(lo - 1, hi + 1)]) for d, (lo, hi) in enumerate(rng)]
        w = [np.array([g.width(d, m) for m in range(lo, hi)]) for d, (lo, hi) in enumerate(rng)]
        sp = [c[d][2:] - c[d][:-2] for d in range(3)]       # x_{m+1} - x_{m-1}
        return _cleaning_metric(self.cart, c, w, sp)

    def clean(self, Unew, G, alpha):
        """Parabolic div B cleaning of a stage result Unew (dict, in place) from
        the ghosted stage input G."""
        D = {leaf: _clib.divb(self.patch(leaf), G[leaf]) for leaf in self.forest.leaves}
        B = self.B
        for leaf in self.forest.leaves:
            Dp = np.full(tuple(b + 2 for b in B[::-1]), np.nan)
            Dp[1:-1, 1:-1, 1:-1] = D[leaf]
            for d in range(3):
                ax = 2 - d
                for side in (0, 1):
                    nbs = self.forest.face_neighbours(leaf, d, side)
                    if len(nbs) != 1 or nbs[0][0] != leaf[0]:
                        continue                        # boundary or level change: no D there
                    src = [slice(None)] * 3
                    src[ax] = slice(B[d] - 1, B[d]) if side == 0 else slice(0, 1)
                    dst = [slice(1, -1)] * 3
                    dst[ax] = slice(0, 1) if side == 0 else slice(B[d] + 1, B[d] + 2)
                    Dp[tuple(dst)] = D[nbs[0]][tuple(src)]
            dx, gs = self._widths(leaf)
            _apply_cleaning(Unew[leaf], G[leaf], Dp, dx, gs, alpha * self.divb_cd)

    def _reflux(self, L, F):
        B = self.B
        for leaf in sorted(self.forest.leaves):
            gc = self.geo[leaf[0]]
            gf = self.geo[leaf[0] + 1] if leaf[0] + 1 < len(self.geo) else None
            for d in range(3):
                for side in (0, 1):
                    nbs = self.forest.face_neighbours(leaf, d, side)
                    if not nbs or nbs[0][0] <= leaf[0]:
                        continue
                    t1, t2 = (d + 1) % 3, (d + 2) % 3
                    nd = 0 if side == 0 else B[d] - 1
                    for a in range(B[t1]):
                        for b in range(B[t2]):
                            loc = [0, 0, 0]
                            loc[d], loc[t1], loc[t2] = nd, a, b
                            glob = [loc[e] + self.cell_range(leaf, e)[0] for e in range(3)]
                            Vc = gc.volume(*glob)
                            acc = np.zeros(self.nv)
                            for ob in (0, 1):
                                for oa in (0, 1):
                                    fg = [0, 0, 0]
                                    fg[t1] = 2 * glob[t1] + oa
                                    fg[t2] = 2 * glob[t2] + ob
                                    # fine cell just across the face, and its face index
                                    fg[d] = 2 * glob[d] + (2 if side else -1)
                                    fw = [int(self._wrap_idx(leaf[0] + 1, e, np.array(fg[e]))) for e in range(3)]
                                    fl = (leaf[0] + 1,) + tuple(fw[e] // B[e] for e in range(3))
                                    floc = [fw[e] - fl[1 + e] * B[e] for e in range(3)]
                                    face_idx = list(floc)
                                    if side == 1:
                                        face_idx[d] = 0        # fine cell's lower face
                                    else:
                                        face_idx[d] = B[d]     # fine cell's upper face
                                    Ff = F[fl][d]
                                    fval = Ff[:, face_idx[2], face_idx[1], face_idx[0]]
                                    Af = gf.area(d, *fw, upper=(side == 0))
                                    acc += Af * fval
                            fidx = list(loc)
                            fidx[d] = B[d] if side else 0
                            Fc = F[leaf][d][:, fidx[2], fidx[1], fidx[0]]
                            am, ap = self.metric(leaf, d, *loc)
                            if side:
                                corr = ap * Fc - acc / Vc
                            else:
                                corr = -am * Fc + acc / Vc
                            L[leaf][:, loc[2], loc[1], loc[0]] += corr

    def max_rate(self, U):
        best = 0.0
        for leaf in self.forest.leaves:
            g = np.zeros((self.nv,) + tuple(b + 4 for b in self.B[::-1]))
            g[:, 2:-2, 2:-2, 2:-2] = U[leaf]
            best = max(best, _clib.max_rate(self.patch(leaf), g))
        return best

    # --- time step ------------------------------------------------------------
    def cfl_dt(self):
        return self.cfl / self.max_rate(self.U)

    def step(self, dt=None, t_end=None):
        """One two-stage step; dt in code units (None = CFL).  Returns dt."""
        if dt is None:
            dt = self.cfl_dt()
            if t_end is not None:
                dt = min(dt, t_end - self.t)
        Un = self.U
        if self.scheme == "hancock":
            L1, G1 = self.predictor(Un, self.t)
        else:
            L1, G1 = self.operator(Un, self.t)
        Us = {b: Un[b] + (0.5 * dt) * L1[b] for b in Un}
        for u in Us.values():
            self.floored += apply_floors(u, self.gamma, self.rho_floor, self.p_floor, self.floor_counts)
        if self.divb_cd > 0.0:
            self.clean(Us, G1, 0.5)
        L2, G2 = self.operator(Us, self.t + 0.5 * dt)
        self.U = {b: Un[b] + dt * L2[b] for b in Un}
        for u in self.U.values():
            self.floored += apply_floors(u, self.gamma, self.rho_floor, self.p_floor, self.floor_counts)
        if self.divb_cd > 0.0:
            self.clean(self.U, G2, 1.0)
        self.t += dt
        self.steps += 1
        return dt

    def advance(self, dt_s, max_steps=10 ** 9):
        t_end = self.t + units.time_code(dt_s)
        n = 0
        while self.t < t_end and n < max_steps:
            self.step(t_end=t_end)
            n += 1
        return n

    # --- refinement ----------------------------------------------------------
    def indicator(self):
        """Per-leaf dict of (E, divv, divscale) arrays on the current state."""
        G = self.ghosted(self.U, self.t)
        out = {}
        a = self.amr
        for leaf in self.forest.leaves:
            er, ev, dv, ds = _clib.indicator(self.patch(leaf), G[leaf], a["eps_lohner"])
            out[leaf] = (a["w_rho"] * er + a["w_v"] * ev, dv, ds)
        return out, G

    def window(self, leaf, cme):
        """Cells inside the refinement windows: |lon - lon_E| <= dlon_E,
        |clt - clt_E| <= dclt_E, |lon - lon_CME| <= dlon_CME (Sect. 3.2)."""
        a = self.amr
        th = self.centres(leaf, 1)[None, :, None]
        ph = self.centres(leaf, 2)[:, None, None]
        if not a.get("use_windows", True) or self.cart:
            return np.ones(self.B[::-1], dtype=bool)

        def wrap(x):
            y = np.mod(x + math.pi, 2 * math.pi) - math.pi
            return np.where(y == -math.pi, math.pi, y)

        w = (np.abs(wrap(ph - math.radians(a["lon_earth_deg"]))) <= math.radians(a["dlon_earth_deg"]))
        w = w & (np.abs(th - math.radians(a["clt_earth_deg"])) <= math.radians(a["dclt_earth_deg"]))
        if cme is not None:
            w = w & (np.abs(wrap(ph - math.radians(cme["lon_deg"]))) <= math.radians(a["dlon_cme_deg"]))
        return np.broadcast_to(w, self.B[::-1])

    def flags(self, ties=None):
        """REFINE / KEEP / COARSEN per leaf (plain criterion).  `ties`, if a
        list, receives (leaf, kind) for cells within the near-tie margins."""
        ind, _ = self.indicator()
        a = self.amr
        crit = a.get("criterion", "shock")
        assert crit in ("shock", "tracer", "combined")
        out = {}
        for leaf, (E, dv, ds) in ind.items():
            win = self.window(leaf, self.cme)
            comp = dv < 0.0
            hot_r = win & comp & (E > a["tol_refine"])
            hot_c = win & comp & (E > a["tol_coarsen"])
            if crit != "shock":
                s = self.U[leaf][8] / self.U[leaf][0]
                tr_r, tr_c = s > a["tracer_refine"], s > a["tracer_coarsen"]
                if crit == "tracer":
                    hot_r, hot_c = tr_r, tr_c
                else:
                    hot_r, hot_c = hot_r | (win & tr_r), hot_c | (win & tr_c)
            if ties is not None:
                for tol in (a["tol_refine"], a["tol_coarsen"]):
                    if np.any(win & comp & (np.abs(E - tol) < 1e-9 * tol)):
                        ties.append((leaf, "E", tol))
                if np.any(win & (E > a["tol_coarsen"] * (1 - 1e-9)) & (np.abs(dv) <= 1e-12 * ds)):
                    ties.append((leaf, "divv", 0.0))
            if leaf[0] < self.max_level and hot_r.any():
                out[leaf] = fo.REFINE
            elif leaf[0] > 1 and not hot_c.any():
                out[leaf] = fo.COARSEN
            else:
                out[leaf] = fo.KEEP
        return out

    def hot(self):
        """Per leaf: 1 if some cell meets the refinement condition (window,
        div V < 0, indicator above tol_refine; Sect. 3.2) whatever the leaf's
        level, else 0."""
        ind, _ = self.indicator()
        out = {}
        for leaf, (E, dv, ds) in ind.items():
            win = self.window(leaf, self.cme)
            out[leaf] = int(bool(np.any(win & (dv < 0.0) & (E > self.amr["tol_refine"]))))
        return out

    def regrid(self, flags=None, buffer_blocks=None):
        """Rebuild the forest from flags (plain criterion if None) and move data."""
        if flags is None:
            flags = self.flags()
        if buffer_blocks is None:
            buffer_blocks = self.amr["buffer_blocks"]
        G = self.ghosted(self.U, self.t)
        new, refined, coarsened = self.forest.regrid(flags, buffer_blocks)
        U = dict(self.U)
        for p in refined:
            for o in range(8):
                ch = (p[0] + 1, 2 * p[1] + (o & 1), 2 * p[2] + ((o >> 1) & 1), 2 * p[3] + ((o >> 2) & 1))
                gidx = [np.arange(ch[1 + d] * self.B[d], (ch[1 + d] + 1) * self.B[d]) for d in range(3)]
                U[ch] = self.prolong(G[p], p, ch[0], gidx)
            del U[p]
        for p in coarsened:
            gidx = [np.arange(p[1 + d] * self.B[d], (p[1 + d] + 1) * self.B[d]) for d in range(3)]
            U[p] = self.restrict(U, p[0], gidx)
            for o in range(8):
                del U[(p[0] + 1, 2 * p[1] + (o & 1), 2 * p[2] + ((o >> 1) & 1), 2 * p[3] + ((o >> 2) & 1))]
        self.forest = fo.Forest(self.nb, self.grid["periodic"], self.max_level, new)
        assert set(U) == new
        self.U = U
        return refined, coarsened

    # --- state exchange ---------------------------------------------------------
    def blocks(self):
        return fo.ordered(self.forest.leaves)

    def state(self):
        """(blocks in (level, Morton) order, stacked U [nb, 8, bk, bj, bi])."""
        bl = self.blocks()
        return bl, np.stack([self.U[b] for b in bl])

    def set_state(self, blocks, U, t_code=None):
        blocks = [tuple(int(x) for x in b) for b in blocks]
        self.forest = fo.Forest(self.nb, self.grid["periodic"], self.max_level, blocks)
        self.U = {b: np.array(U[n], dtype=np.float64) for n, b in enumerate(blocks)}
        if t_code is not None:
            self.t = t_code

    def total(self):
        """sum over leaves of V U per conserved variable."""
        tot = np.zeros(self.nv)
        for leaf, u in self.U.items():
            g = self.geo[leaf[0]]
            r = [self.cell_range(leaf, d) for d in range(3)]
            wi = np.array([g.volume_weight(0, x) for x in range(*r[0])])
            wj = np.array([g.volume_weight(1, x) for x in range(*r[1])])
            wk = np.array([g.volume_weight(2, x) for x in range(*r[2])])
            V = wk[:, None, None] * wj[None, :, None] * wi[None, None, :]
            tot += (u * V).reshape(self.nv, -1).sum(axis=1)
        return tot

    # --- sampling ---------------------------------------------------------------
    def _cell_value(self, level, gidx):
        """Conserved value of global cell gidx at `level`: the leaf cell if a
        leaf of that level holds it, the covering coarse cell if coarser, the
        volume-weighted mean of its children if finer."""
        leaf_idx = tuple(gidx[d] // self.B[d] for d in range(3))
        c = self.forest.covering_leaf(level, leaf_idx)
        if c is not None:
            s = 2 ** (level - c[0])
            cg = [gidx[d] // s for d in range(3)]
            loc = [cg[d] - c[1 + d] * self.B[d] for d in range(3)]
            return self.U[c][:, loc[2], loc[1], loc[0]]
        g = self.geo[level + 1]
        num, den = np.zeros(self.nv), 0.0
        for o in range(8):
            ch = (2 * gidx[0] + (o & 1), 2 * gidx[1] + ((o >> 1) & 1), 2 * gidx[2] + ((o >> 2) & 1))
            w = g.volume_weight(0, ch[0]) * g.volume_weight(1, ch[1]) * g.volume_weight(2, ch[2])
            num += w * self._cell_value(level + 1, ch)
            den += w
        return num / den

    def sample(self, r_au, colat_deg, lon_deg):
        """Trilinear interpolation of primitives between the cell centres of
        the level of the finest leaf containing the point (code units)."""
        x = [r_au, math.radians(colat_deg), math.radians(lon_deg)] if not self.cart \
            else [r_au, colat_deg, lon_deg]
        g1 = self.geo[1]
        # leaf containing the point
        lvl = None
        for level in range(self.max_level, 0, -1):
            g = self.geo[level]
            idx = []
            for d in range(3):
                f = g.f[d][2:g.n[d] + 3]
                m = int(np.searchsorted(f, x[d], side="right") - 1)
                m = min(max(m, 0), g.n[d] - 1)
                idx.append(m)
            if (level,) + tuple(idx[d] // self.B[d] for d in range(3)) in self.forest.leaves:
                lvl = level
                break
        if lvl is None:
            raise ValueError("point outside the domain")
        del g1
        g = self.geo[lvl]
        lo, wt = [], []
        for d in range(3):
            c = 0.5 * (g.f[d][2:g.n[d] + 2] + g.f[d][3:g.n[d] + 3])
            if self.grid["periodic"][d]:
                period = g.f[d][g.n[d] + 2] - g.f[d][2]
                xx = (x[d] - c[0]) % period + c[0]
                m = int(np.searchsorted(c, xx, side="right") - 1)
                if m >= g.n[d] - 1:
                    c_hi = c[0] + period
                    lo.append(m)
                    wt.append((xx - c[m]) / (c_hi - c[m]))
                else:
                    lo.append(m)
                    wt.append((xx - c[m]) / (c[m + 1] - c[m]))
            else:
                m = int(np.searchsorted(c, x[d], side="right") - 1)
                if m < 0:
                    lo.append(0); wt.append(0.0)
                elif m >= g.n[d] - 1:
                    lo.append(g.n[d] - 2); wt.append(1.0)
                else:
                    lo.append(m); wt.append((x[d] - c[m]) / (c[m + 1] - c[m]))
        out = np.zeros(self.nv)
        for o in range(8):
            off = (o & 1, (o >> 1) & 1, (o >> 2) & 1)
            gi = []
            w = 1.0
            for d in range(3):
                m = lo[d] + off[d]
                if self.grid["periodic"][d]:
                    m %= g.n[d]
                gi.append(m)
                w *= wt[d] if off[d] else (1.0 - wt[d])
            u = self._cell_value(lvl, gi)
            out += w * boundary.cons_to_prims(u.reshape(self.nv, 1), self.gamma)[:, 0]
        return out


class PatchSolver:
    """Single-level solver on one global ghosted patch (no blocks).  Used as
    an independent check of the block decomposition and as the CPU baseline."""

    def __init__(self, grid, wind=None, cme=None, omega=None, gm=None, t0_s=0.0, initial="wind",
                 rho_floor=RHO_FLOOR, p_floor=P_FLOOR, limiter="mc", scheme="two_stage", divb_cd=0.0,
                 tracer=False):
        self.rho_floor, self.p_floor, self.floored = rho_floor, p_floor, 0
        self.limiter, self.scheme, self.divb_cd = limiter, scheme, float(divb_cd)
        self.nv = 9 if tracer else NV
        assert scheme in ("two_stage", "hancock")
        self.floor_counts = [0, 0]         # density-floored, pressure-floored cells
        self.grid = dict(grid)
        self.grid.setdefault("geometry", "spherical")
        self.grid.setdefault("periodic", (False, False, False))
        self.grid.setdefault("stretched_r", False)
        self.cart = self.grid["geometry"] == "cartesian"
        self.gamma = float(self.grid.get("gamma", 1.5))
        self.cfl = float(self.grid.get("cfl", 0.4))
        self.omega, self.gm = _phys(self.grid, omega, gm)
        self.bc = _bc_of(self.grid)
        self.wind, self.cme = wind, cme
        self.geo = geometry.LevelGeometry(self.grid, 1)
        self.n = self.geo.n
        self.r_in = self.geo.f[0][2]
        self.pg = _clib.PatchGeom(self.geo.f[0], self.geo.f[1], self.geo.f[2], self.cart,
                                  self.gamma, self.omega, self.gm, limiter, self.nv)
        self.t = units.time_code(t0_s)
        ni, nj, nk = self.n
        if initial == "wind" and wind is not None and not self.cart:
            r = np.array([self.geo.centre(0, i) for i in range(ni)])[None, None, :]
            th = np.array([self.geo.centre(1, j) for j in range(nj)])[None, :, None]
            ph = np.array([self.geo.centre(2, k) for k in range(nk)])[:, None, None]
            W = boundary.initial_prims(wind, r, th, ph, self.r_in, self.omega, self.gamma)
            if self.nv > NV:
                W = np.concatenate([W, np.zeros((1,) + W.shape[1:])])
            self.U = boundary.prims_to_cons(W, self.gamma)
        else:
            self.U = np.zeros((self.nv, nk, nj, ni))

    def ghosted(self, U, t):
        ni, nj, nk = self.n
        G = np.zeros((self.nv, nk + 4, nj + 4, ni + 4))
        G[:, 2:-2, 2:-2, 2:-2] = U
        n = self.n
        for d in range(3):
            ax = 3 - d
            for side in (0, 1):
                kind = self.bc[d][side]
                dst = [slice(None), slice(2, 2 + nk), slice(2, 2 + nj), slice(2, 2 + ni)]
                dst[ax] = slice(0, 2) if side == 0 else slice(2 + n[d], 4 + n[d])
                src = list(dst)
                if kind == "periodic":
                    cells = (np.array([-2, -1]) if side == 0 else np.array([n[d], n[d] + 1])) % n[d]
                    src[ax] = cells + 2
                    G[tuple(dst)] = G[tuple(src)]
                elif kind == "outflow":
                    e = 2 if side == 0 else 1 + n[d]
                    src[ax] = slice(e, e + 1)
                    G[tuple(dst)] = G[tuple(src)]
                elif kind == "inner":
                    th = np.array([self.geo.centre(1, j) for j in range(nj)])[None, :]
                    ph = np.array([self.geo.centre(2, k) for k in range(nk)])[:, None]
                    W = boundary.boundary_prims(self.wind, self.cme, th + 0.0 * ph, ph + 0.0 * th,
                                                self.r_in, self.omega, t)
                    if self.nv > NV:
                        s_in = boundary.cme_mask(self.cme, th + 0.0 * ph, ph + 0.0 * th, self.r_in, t) \
                            if self.cme is not None else np.zeros(W.shape[1:], dtype=bool)
                        W = np.concatenate([W, s_in[None].astype(np.float64)])
                    G[tuple(dst)] = boundary.prims_to_cons(W, self.gamma)[:, :, :, None]
                else:
                    raise ValueError(kind)
        return G

    def operator(self, U, t):
        G = self.ghosted(U, t)
        L, _, bad = _clib.rhs(self.pg, G)
        if bad:
            raise UnphysicalState("%d unphysical cells" % bad)
        return L

    def predictor(self, U, t):
        L, bad = _clib.rhs_hancock(self.pg, self.ghosted(U, t))
        if bad:
            raise UnphysicalState("%d unphysical cells" % bad)
        return L

    def clean(self, Unew, Uin, t, alpha):
        """Parabolic div B cleaning of Unew (in place) from the stage input Uin
        (ghosts at t): the forest form on one patch; periodic directions wrap."""
        G = self.ghosted(Uin, t)
        D = _clib.divb(self.pg, G)
        Dp = np.pad(D, 1, mode="constant", constant_values=np.nan)
        for d in range(3):
            if self.bc[d][0] == "periodic":
                ax = 2 - d
                lo, hi = [slice(1, -1)] * 3, [slice(1, -1)] * 3
                src_lo, src_hi = [slice(None)] * 3, [slice(None)] * 3
                lo[ax], hi[ax] = slice(0, 1), slice(-1, None)
                src_lo[ax], src_hi[ax] = slice(-1, None), slice(0, 1)
                Dp[tuple(lo)] = D[tuple(src_lo)]
                Dp[tuple(hi)] = D[tuple(src_hi)]
        g = self.geo
        c = [geometry.centres(g.f[d])[1:-1] for d in range(3)]      # cells -1 .. n
        w = [np.diff(g.f[d])[2:-2] for d in range(3)]
        sp = [c[d][2:] - c[d][:-2] for d in range(3)]
        dx, gs = _cleaning_metric(self.cart, c, w, sp)
        _apply_cleaning(Unew, G, Dp, dx, gs, alpha * self.divb_cd)

    def cfl_dt(self):
        G = np.zeros((self.nv,) + tuple(x + 4 for x in self.n[::-1]))
        G[:, 2:-2, 2:-2, 2:-2] = self.U
        return self.cfl / _clib.max_rate(self.pg, G)

    def step(self, dt=None):
        if dt is None:
            dt = self.cfl_dt()
        Un = self.U
        L1 = self.predictor(Un, self.t) if self.scheme == "hancock" else self.operator(Un, self.t)
        Us = Un + (0.5 * dt) * L1
        self.floored += apply_floors(Us, self.gamma, self.rho_floor, self.p_floor, self.floor_counts)
        if self.divb_cd > 0.0:
            self.clean(Us, Un, self.t, 0.5)
        L2 = self.operator(Us, self.t + 0.5 * dt)
        self.U = Un + dt * L2
        self.floored += apply_floors(self.U, self.gamma, self.rho_floor, self.p_floor, self.floor_counts)
        if self.divb_cd > 0.0:
            self.clean(self.U, Us, self.t + 0.5 * dt, 1.0)
        self.t += dt
        return dt

    def total(self):
        g = self.geo
        ni, nj, nk = self.n
        wi = np.array([g.volume_weight(0, x) for x in range(ni)])
        wj = np.array([g.volume_weight(1, x) for x in range(nj)])
        wk = np.array([g.volume_weight(2, x) for x in range(nk)])
        V = wk[:, None, None] * wj[None, :, None] * wi[None, None, :]
        return (self.U * V).reshape(self.nv, -1).sum(axis=1)

    def to_blocks(self, block):
        """Split the patch state into base-level blocks, (level, Morton) order."""
        nb = [self.n[d] // block[d] for d in range(3)]
        leaves = [(1, i, j, k) for k in range(nb[2]) for j in range(nb[1]) for i in range(nb[0])]
        leaves = fo.ordered(leaves)
        out = []
        for b in leaves:
            out.append(self.U[:, b[3] * block[2]:(b[3] + 1) * block[2],
                              b[2] * block[1]:(b[2] + 1) * block[1],
                              b[1] * block[0]:(b[1] + 1) * block[0]])
        return leaves, np.stack(out)
