"""Block-AMR forest of the oracle (test infrastructure only).

Paper Sect. 3: refinement splits a block's cells in two in every direction;
adjacent blocks differ by at most one level; blocks coarsen once the
criterion no longer holds.  A leaf is (level, i, j, k), level >= 1, with
(i, j, k) its block index on that level (level l has nb * 2^(l-1) blocks per
direction).

Regrid steps (each written as plain set logic):
  1. clamp: REFINE at the maximum level and COARSEN at level 1 become KEEP;
  2. buffer: every leaf touching a REFINE leaf across one of its six faces
     becomes REFINE (buffer on, level permitting, not finer than the REFINE
     leaf) or is at least kept from coarsening;
  3. 2:1 closure to a fixpoint: a leaf one level coarser than a REFINE leaf
     and touching it across any face, edge or corner becomes REFINE;
  4. coarsening: eight sibling leaves that are all COARSEN (after 2 and 3)
     merge into their parent, unless the parent would touch a leaf two or more
     levels finer in the forest after refinement; at most one level per regrid;
  5. the new leaf set; data moves are prolongation into new children and
     restriction into new parents.
"""
REFINE, KEEP, COARSEN = 1, 0, -1


class Forest:
    def __init__(self, nb, periodic, max_level, leaves=None):
        self.nb = tuple(int(x) for x in nb)
        self.periodic = tuple(bool(p) for p in periodic)
        self.max_level = int(max_level)
        if leaves is None:
            leaves = [(1, i, j, k) for k in range(nb[2]) for j in range(nb[1]) for i in range(nb[0])]
        self.leaves = set(tuple(b) for b in leaves)

    # --- index helpers ----------------------------------------------------
    def nblocks(self, level):
        f = 2 ** (level - 1)
        return tuple(n * f for n in self.nb)

    def wrap(self, level, idx):
        """Wrap a block index at `level` through periodic directions; None if outside."""
        n = self.nblocks(level)
        out = []
        for d in range(3):
            x = idx[d]
            if self.periodic[d]:
                x %= n[d]
            elif x < 0 or x >= n[d]:
                return None
            out.append(x)
        return tuple(out)

    def covering_leaf(self, level, idx):
        """Leaf containing the region of block idx at `level` (itself or an
        ancestor), or None if that region is refined further."""
        l, c = level, tuple(idx)
        while l >= 1:
            if (l,) + c in self.leaves:
                return (l,) + c
            l -= 1
            c = tuple(x // 2 for x in c)
        return None

    def face_neighbours(self, leaf, d, side):
        """Leaves across face (d, side) of `leaf`: [] at a physical boundary,
        [same-level or coarser leaf], or the finer leaves touching the face."""
        l = leaf[0]
        idx = list(leaf[1:])
        idx[d] += 1 if side else -1
        w = self.wrap(l, idx)
        if w is None:
            return []
        c = self.covering_leaf(l, w)
        if c is not None:
            return [c]
        out = []
        # region is refined: the children adjacent to the face (recursively)
        stack = [(l, w)]
        while stack:
            lv, bi = stack.pop()
            for o in range(8):
                off = (o & 1, (o >> 1) & 1, (o >> 2) & 1)
                if off[d] != (0 if side else 1):
                    continue
                ch = (lv + 1,) + tuple(2 * bi[e] + off[e] for e in range(3))
                if ch in self.leaves:
                    out.append(ch)
                else:
                    stack.append((lv + 1, ch[1:]))
        return sorted(out)

    def extent(self, leaf, fine_level):
        """Half-open extent of a leaf in block units of `fine_level`."""
        s = 2 ** (fine_level - leaf[0])
        return [(leaf[1 + d] * s, (leaf[1 + d] + 1) * s) for d in range(3)]

    def touch(self, a, b):
        """True if the closures of leaves a and b intersect (face, edge or
        corner contact or overlap), through periodic directions."""
        L = max(a[0], b[0], self.max_level)
        ea, eb = self.extent(a, L), self.extent(b, L)
        n = self.nblocks(L)
        for d in range(3):
            shifts = (-n[d], 0, n[d]) if self.periodic[d] else (0,)
            if not any(ea[d][0] <= eb[d][1] + s and eb[d][0] + s <= ea[d][1] for s in shifts):
                return False
        return True

    def leaves_touching_at_level(self, leaf, level):
        """Leaves at exactly `level` whose closure touches `leaf`."""
        out = []
        L = leaf[0]
        if level <= L:
            s = 2 ** (L - level)
            base = [leaf[1 + d] // s for d in range(3)]
            rng = [range(base[d] - 1, base[d] + 2) for d in range(3)]
        else:
            s = 2 ** (level - L)
            rng = [range(leaf[1 + d] * s - 1, (leaf[1 + d] + 1) * s + 1) for d in range(3)]
        seen = set()
        for k in rng[2]:
            for j in rng[1]:
                for i in rng[0]:
                    w = self.wrap(level, (i, j, k))
                    if w is None:
                        continue
                    c = (level,) + w
                    if c in self.leaves and c != leaf and c not in seen and self.touch(leaf, c):
                        seen.add(c)
                        out.append(c)
        return sorted(out)

    # --- regrid -------------------------------------------------------------
    def regrid(self, flags, buffer_blocks=1):
        """Apply per-leaf flags {leaf: REFINE/KEEP/COARSEN}.
        Returns (new_leaves, refined, coarsened_parents)."""
        f = {b: flags.get(b, KEEP) for b in self.leaves}
        for b in self.leaves:
            if f[b] == REFINE and b[0] >= self.max_level:
                f[b] = KEEP
            if f[b] == COARSEN and b[0] <= 1:
                f[b] = KEEP
        # 2. buffer
        for b in sorted(x for x in self.leaves if f[x] == REFINE):
            for d in range(3):
                for side in (0, 1):
                    for n in self.face_neighbours(b, d, side):
                        if buffer_blocks and n[0] < self.max_level and n[0] <= b[0]:
                            f[n] = REFINE
                        elif f[n] == COARSEN:
                            f[n] = KEEP
        # 3. 2:1 closure
        changed = True
        while changed:
            changed = False
            for b in sorted(x for x in self.leaves if f[x] == REFINE):
                if b[0] < 2:
                    continue
                for n in self.leaves_touching_at_level(b, b[0] - 1):
                    if f[n] != REFINE:
                        f[n] = REFINE
                        changed = True
        refined = sorted(b for b in self.leaves if f[b] == REFINE)
        post = set(self.leaves)
        for b in refined:
            post.discard(b)
            for o in range(8):
                post.add((b[0] + 1, 2 * b[1] + (o & 1), 2 * b[2] + ((o >> 1) & 1), 2 * b[3] + ((o >> 2) & 1)))
        # 4. coarsening
        parents = {}
        for b in self.leaves:
            if f[b] == COARSEN:
                p = (b[0] - 1, b[1] // 2, b[2] // 2, b[3] // 2)
                parents.setdefault(p, []).append(b)
        post_forest = Forest(self.nb, self.periodic, self.max_level, post)
        coarsened = []
        for p in sorted(parents):
            if len(parents[p]) != 8:
                continue
            ok = True
            for lv in range(p[0] + 2, self.max_level + 1):
                if post_forest.leaves_touching_at_level(p, lv):
                    ok = False
                    break
            if ok:
                coarsened.append(p)
        new = set(post)
        for p in coarsened:
            for c in parents[p]:
                new.discard(c)
            new.add(p)
        return new, refined, coarsened

    def check_balance(self):
        """2:1 over all 26 directions and proper nesting (no overlaps)."""
        for b in self.leaves:
            # no ancestor is also a leaf
            l, c = b[0] - 1, b[1:]
            while l >= 1:
                c = tuple(x // 2 for x in c)
                if (l,) + c in self.leaves:
                    return False
                l -= 1
            for lv in range(b[0] + 2, self.max_level + 2):
                if self.leaves_touching_at_level(b, lv):
                    return False
        return True


def morton(i, j, k):
    """Bit-interleaved key, i in the lowest bit of each triple."""
    key = 0
    for bit in range(21):
        key |= ((i >> bit) & 1) << (3 * bit)
        key |= ((j >> bit) & 1) << (3 * bit + 1)
        key |= ((k >> bit) & 1) << (3 * bit + 2)
    return key


def ordered(leaves):
    """Leaves in ascending (level, Morton) order."""
    return sorted(leaves, key=lambda b: (b[0], morton(b[1], b[2], b[3])))
