"""Mesh geometry of the oracle (test infrastructure only).

Paper Sect. 2.2: radial stretching keeps cells cubical; the number of radial
cells follows Eq. (5), N = log(r_out/r_in) / log((2 + dtheta)/(2 - dtheta)).
With that ratio q, consecutive radial faces grow geometrically, r_{k+1} = q r_k,
which is the statement dr = r_c dtheta for a cell of centre r_c = (r_k+r_{k+1})/2.

Here a level-l grid with N_l radial cells uses faces
    r_k = r_in exp(k ln(r_out/r_in) / N_l),  k = -2 .. N_l + 2
(the two ghost faces on each side continue the progression; r_{N_l} is set
to r_out exactly), or r_k = r_in + k (r_out - r_in)/N_l on an equidistant
grid.  Angles are uniform.  Refinement level l has N_l = N_1 2^(l-1) cells
per direction (Sect. 3: each level halves the cells in all directions), so a
child splits its parent at the geometric midpoint in r.
"""
import math

import numpy as np

from . import units


def stretched_cell_count(r_in, r_out, dtheta):
    """Eq. (5): optimal radial cell count for angular resolution dtheta [rad]."""
    return math.log(r_out / r_in) / math.log((2.0 + dtheta) / (2.0 - dtheta))


def radial_faces(r_in, r_out, n, stretched):
    k = np.arange(-2, n + 3, dtype=np.float64)
    if stretched:
        lg = math.log(r_out / r_in)
        f = np.array([r_in * math.exp(kk * (lg / n)) for kk in k])
    else:
        h = (r_out - r_in) / n
        f = np.array([r_in + kk * h for kk in k])
    f[n + 2] = r_out
    f[2] = r_in
    return f


def uniform_faces(x0, x1, n):
    h = (x1 - x0) / n
    f = np.array([x0 + kk * h for kk in range(-2, n + 3)], dtype=np.float64)
    f[n + 2] = x1
    f[2] = x0
    return f


def centres(f):
    return 0.5 * (f[:-1] + f[1:])


class LevelGeometry:
    """Face arrays (with two ghost faces each side) of one refinement level.

    Spherical: direction 0 = r [AU], 1 = colatitude theta [rad], 2 = longitude
    phi [rad].  Cartesian: x, y, z in code units.
    """

    def __init__(self, grid, level):
        self.level = level
        fac = 2 ** (level - 1)
        self.n = tuple(int(c) * fac for c in grid["n"])
        self.cartesian = grid["geometry"] == "cartesian"
        x0, x1 = grid["x0"], grid["x1"]
        if self.cartesian:
            self.f = [uniform_faces(x0[d], x1[d], self.n[d]) for d in range(3)]
        else:
            self.f = [radial_faces(x0[0], x1[0], self.n[0], grid["stretched_r"]),
                      uniform_faces(math.radians(x0[1]), math.radians(x1[1]), self.n[1]),
                      uniform_faces(math.radians(x0[2]), math.radians(x1[2]), self.n[2])]

    def faces(self, d, lo, hi):
        """Faces of cells lo..hi-1 with two ghost faces each side (lo-2 .. hi+2)."""
        return np.ascontiguousarray(self.f[d][lo:hi + 5])

    def centre(self, d, m):
        return 0.5 * (self.f[d][m + 2] + self.f[d][m + 3])

    def width(self, d, m):
        return self.f[d][m + 3] - self.f[d][m + 2]

    def volume_weight(self, d, m):
        """Factor of the cell volume that depends on direction d only."""
        a, b = self.f[d][m + 2], self.f[d][m + 3]
        if self.cartesian:
            return b - a
        if d == 0:
            return (b ** 3 - a ** 3) / 3.0
        if d == 1:
            return math.cos(a) - math.cos(b)
        return b - a

    def volume(self, i, j, k):
        return self.volume_weight(0, i) * self.volume_weight(1, j) * self.volume_weight(2, k)

    def area(self, d, i, j, k, upper):
        """Full area of the lower (upper=False) or upper face along d of cell (i, j, k)."""
        f = self.f
        idx = (i, j, k)
        m = idx[d] + (1 if upper else 0)
        if self.cartesian:
            a = 1.0
            for e in range(3):
                if e != d:
                    a *= self.width(e, idx[e])
            return a
        rm, rp = f[0][i + 2], f[0][i + 3]
        tm, tp = f[1][j + 2], f[1][j + 3]
        pm, pp = f[2][k + 2], f[2][k + 3]
        if d == 0:
            r = f[0][m + 2]
            return r * r * (math.cos(tm) - math.cos(tp)) * (pp - pm)
        if d == 1:
            t = f[1][m + 2]
            return 0.5 * (rp * rp - rm * rm) * math.sin(t) * (pp - pm)
        return 0.5 * (rp * rp - rm * rm) * (tp - tm)


def width_at_radius_rsun(r_in, r_out, n, r):
    """Radial width in solar radii of the stretched cell centred on radius r:
    r (q^(1/2) - q^(-1/2)), q = (r_out/r_in)^(1/n)."""
    q = (r_out / r_in) ** (1.0 / n)
    return r * (math.sqrt(q) - 1.0 / math.sqrt(q)) * units.AU_IN_RSUN
