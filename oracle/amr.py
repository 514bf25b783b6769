"""Octree AMR mesh for the DG oracle (test infrastructure only).

Sec. 4.4: cubic cells in an octree, each refinement splitting a cell into
2^D children; all levels advance with one global time step.  The paper
defers the hanging-face treatment to Schaal et al. (2015); the reading used
here is the L2 one: on a face between a coarse cell and its 2^(D-1) finer
neighbours the flux is evaluated at the Gauss-Legendre points of each fine
face, the coarse trace being evaluated there (prolongation of the coarse
trace), and the coarse cell integrates the same fluxes with weights
w_r / 2^(D-1) (restriction onto the coarse face), so the scheme stays
conservative.

A leaf is (level, i, j[, k]) with integer coordinates on the level grid of
n0 * 2^level cells per axis of the periodic box [0, box]^D.  Faces are listed
once, from the left cell's +e_a side: same level (both full), a finer right
region (one face per fine neighbour, the coarse left side on quarter j), or
a coarser right cell (fine left side full, the coarse right side on quarter
j).  Quarter index j has bit t set when the fine face lies in the upper half
of the t-th tangential axis (tangential axes in increasing order).
"""
import numpy as np

from .dg import Mesh


def morton_key(level, ijk, lmax):
    """Morton (Z-order) key of a leaf at the finest level lmax."""
    s = lmax - level
    c = [int(x) << s for x in ijk]
    key = 0
    bits = max(1, max(c).bit_length() if max(c) > 0 else 1)
    for b in range(bits + 1):
        for a, x in enumerate(c):
            key |= ((x >> b) & 1) << (b * len(c) + a)
    return key


class Octree:
    """Leaves of a periodic octree (quadtree in 2-D)."""

    def __init__(self, D, n0, leaves, box=1.0):
        self.D, self.n0, self.box = D, n0, box
        self.leaves = [(int(l), tuple(int(x) for x in c)) for l, c in leaves]
        self.index = {lf: i for i, lf in enumerate(self.leaves)}
        if len(self.index) != len(self.leaves):
            raise ValueError("duplicate leaves")

    @staticmethod
    def uniform(D, n0, box=1.0):
        import itertools
        return Octree(D, n0, [(0, c[::-1]) for c in itertools.product(range(n0), repeat=D)], box)

    def ncell(self, level):
        return self.n0 << level

    def wrap(self, level, c):
        m = self.ncell(level)
        return tuple(x % m for x in c)

    def is_leaf(self, level, c):
        return (level, self.wrap(level, c)) in self.index

    def morton_sorted(self):
        lmax = max(l for l, _ in self.leaves)
        order = sorted(range(len(self.leaves)), key=lambda i: morton_key(*self.leaves[i], lmax))
        return Octree(self.D, self.n0, [self.leaves[i] for i in order], self.box)

    @staticmethod
    def from_arrays(D, n0, level, ijk, box=1.0):
        return Octree(D, n0, [(int(l), tuple(int(x) for x in c[:D])) for l, c in zip(level, ijk)], box)

    # ------------------------------------------------------------------
    def refine(self, flags):
        """New octree with the flagged leaves split into 2^D children."""
        out = []
        D = self.D
        for (l, c), f in zip(self.leaves, flags):
            if not f:
                out.append((l, c))
                continue
            for off in range(1 << D):
                out.append((l + 1, tuple(2 * c[a] + ((off >> a) & 1) for a in range(D))))
        return Octree(D, self.n0, out, self.box)

    def balance_violations(self):
        """Leaves with a face neighbour more than one level finer (2:1 rule)."""
        bad = np.zeros(len(self.leaves), dtype=bool)
        for i, (l, c) in enumerate(self.leaves):
            for a in range(self.D):
                for s in (-1, 1):
                    nc = list(c)
                    nc[a] += s
                    nc = tuple(nc)
                    if self.is_leaf(l, nc):
                        continue
                    if l > 0 and self.is_leaf(l - 1, tuple(x // 2 for x in self.wrap(l, nc))):
                        continue
                    # finer region: all children adjacent to this face must be leaves
                    for ch in self._adjacent_children(l, nc, a, s):
                        if not self.is_leaf(l + 1, ch):
                            bad[i] = True
        return bad

    def balanced(self):
        t = self
        for _ in range(20):
            bad = t.balance_violations()
            if not bad.any():
                return t
            t = t.refine(bad)
        raise RuntimeError("2:1 balance did not converge")

    def _adjacent_children(self, l, nc, a, s):
        """Children (level l+1) of region nc touching the face shared with the
        cell on side -s along a."""
        D = self.D
        nc = self.wrap(l, nc)
        tang = [b for b in range(D) if b != a]
        out = []
        for q in range(1 << (D - 1)):
            ch = [0] * D
            ch[a] = 2 * nc[a] + (0 if s > 0 else 1)
            for j, b in enumerate(tang):
                ch[b] = 2 * nc[b] + ((q >> j) & 1)
            out.append(tuple(ch))
        return out

    # ------------------------------------------------------------------
    def mesh(self):
        """oracle Mesh with cell sizes, centres and the face list."""
        D = self.D
        C = len(self.leaves)
        h = np.array([self.box / self.ncell(l) for l, _ in self.leaves])
        centers = np.array([[(c[a] + 0.5) * self.box / self.ncell(l) for a in range(D)] for l, c in self.leaves])
        faces = []
        for a in range(D):
            tang = [b for b in range(D) if b != a]
            L, R, sL, sR = [], [], [], []
            for i, (l, c) in enumerate(self.leaves):
                nc = list(c)
                nc[a] += 1
                nc = self.wrap(l, tuple(nc))
                if (l, nc) in self.index:
                    L.append(i); R.append(self.index[(l, nc)]); sL.append(-1); sR.append(-1)
                    continue
                if l > 0 and (l - 1, tuple(x // 2 for x in nc)) in self.index:
                    # coarser right cell: our face is quarter j of its -a face
                    j = sum(((c[b] & 1) << k) for k, b in enumerate(tang))
                    L.append(i); R.append(self.index[(l - 1, tuple(x // 2 for x in nc))]); sL.append(-1); sR.append(j)
                    continue
                for q, ch in enumerate(self._adjacent_children(l, nc, a, +1)):
                    if (l + 1, ch) not in self.index:
                        raise ValueError("mesh is not 2:1 balanced")
                    L.append(i); R.append(self.index[(l + 1, ch)]); sL.append(q); sR.append(-1)
            faces.append(dict(axis=a, L=np.array(L), R=np.array(R), subL=np.array(sL), subR=np.array(sR)))
        m = Mesh(D, h, centers, faces)
        m.box = self.box
        m.octree = self
        return m

    def levels(self):
        return np.array([l for l, _ in self.leaves], dtype=np.int8)

    def coords(self):
        return np.array([list(c) + [0] * (3 - self.D) for _, c in self.leaves], dtype=np.int32)
