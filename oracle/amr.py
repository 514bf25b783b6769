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
        """Leaves with a face neighbour more than one level finer (2:1 rule).
        A leaf whose neighbour is coarser (by any number of levels) is not in
        violation itself: the coarser side is, and refining it is what
        restores the rule."""
        bad = np.zeros(len(self.leaves), dtype=bool)
        for i, (l, c) in enumerate(self.leaves):
            for a in range(self.D):
                for s in (-1, 1):
                    nc = list(c)
                    nc[a] += s
                    nc = self.wrap(l, tuple(nc))
                    if any(self.is_leaf(l - k, tuple(x >> k for x in nc)) for k in range(l + 1)):
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


# ----------------------------------------------------------------------
# Dynamic refinement (Sec. 4.4): smoothness indicator, L2 prolongation and
# restriction of the modal weights, and the regrid of a leaf set.

from functools import lru_cache  # noqa: E402

from . import basis as B  # noqa: E402
from . import physics as ph  # noqa: E402
from .quadrature import tensor_rule  # noqa: E402


@lru_cache(maxsize=None)
def _scalar_polys(D, d):
    """Exact polynomials of the Legendre modes (3-variable exponents)."""
    return tuple(B._legendre_product_poly(tuple(e) + (0,) * (3 - D)) for e in B.mode_exponents(D, d))


def _kth_derivative_values(p, a, k, xi):
    for _ in range(k):
        p = B._pderiv(p, a)
    return B._peval(p, xi)


def smoothness(s, w, fields=(ph.RHO, ph.B1, ph.B2, ph.B3)):
    """S_alpha(u) = sum_{k=1}^{d} 2^(2k-1) int_{[-1,1]^D} (d^k u / d xi_alpha^k)^2
    (the smoothness indicator of Sec. 4.4, on the reference cell) for each
    cell, monitored field and direction: array [C, len(fields), D].  The
    field's polynomial is its Legendre expansion, or for B under the Powell
    scheme its component of the LDF expansion; the integrals are exact with
    the (d+1)-point Gauss rule (integrands of degree <= 2(d - k))."""
    D, d, n = s.D, s.d, s.n
    xq, wq = tensor_rule(d + 1, D)
    xq3 = np.concatenate([xq, np.zeros((xq.shape[0], 3 - D))], axis=1)
    C = w.shape[0]
    out = np.zeros((C, len(fields), D))
    leg = _scalar_polys(D, d)
    ldf = B.ldf_basis_exact(D, d)[0] if s.nldf else None
    for i, v in enumerate(fields):
        if v in s.leg_vars:
            j = s.leg_vars.index(v)
            polys = leg
            wv = w[:, j * n:(j + 1) * n]
        else:
            c = v - ph.B1
            polys = [V[c] for V in ldf]
            wv = w[:, len(s.leg_vars) * n:]
        for a in range(D):
            for k in range(1, d + 1):
                T = np.stack([_kth_derivative_values(p, a, k, xq3) for p in polys], axis=1)  # [Q, modes]
                du = wv @ T.T                                                           # [C, Q]
                out[:, i, a] += 2.0 ** (2 * k - 1) * (du ** 2 * wq).sum(axis=1)
    return out


def _octant_shift(o, D):
    return np.array([2 * ((o >> a) & 1) - 1 for a in range(D)], dtype=np.float64)


def prolong(s, wp, o):
    """Weights of child o (bit a of o: upper half along axis a) of a cell with
    weights wp: the L2 projection of the parent's polynomial restricted to
    the octant onto the child's basis (exact: the same polynomial)."""
    xq, wq = tensor_rule(s.d + 1, s.D)
    xi_p = 0.5 * (xq + _octant_shift(o, s.D))
    U = s.nodal(np.asarray(wp)[None, :], xi=xi_p)
    return s.project_test(U, s._basis_at(xq), wq)[0] / s.M


def restrict(s, wc):
    """Weights of the parent of the 2^D children wc[o] (octant order): the L2
    projection of the piecewise polynomial onto the parent's basis; each
    octant contributes with the Jacobian 2^-D of the map to the parent's
    reference cell."""
    xq, wq = tensor_rule(s.d + 1, s.D)
    acc = np.zeros(s.nmodes)
    for o in range(1 << s.D):
        U = s.nodal(np.asarray(wc[o])[None, :], xi=xq)
        xi_p = 0.5 * (xq + _octant_shift(o, s.D))
        acc += s.project_test(U, s._basis_at(xi_p), wq * 2.0 ** (-s.D))[0]
    return acc / s.M


def _octant_of(c, D):
    return sum((c[a] & 1) << a for a in range(D))


def regrid(tree, s, w, s_tilde=0.03, fields=(ph.RHO, ph.B1, ph.B2, ph.B3), max_level=8):
    """One regrid of Sec. 4.4.  A leaf is refined when S_alpha(u) > 2 S~ for
    any monitored field and direction (and its level is below max_level); a
    complete group of 2^D sibling leaves, none of them marked for refinement,
    is merged into its parent when the parent's polynomial (the restriction
    of the children) has S_alpha(u) < S~/2 for every field and direction.
    2:1 balance: a merge that would leave a face neighbour two levels finer
    is dropped; remaining violations are removed by refinement.  Returns
    (new tree, new weights, stats)."""
    D = tree.D
    Sv = smoothness(s, w, fields)
    refine = (Sv > 2.0 * s_tilde).reshape(len(tree.leaves), -1).any(axis=1)
    refine &= np.array([l < max_level for l, _ in tree.leaves])
    # complete sibling groups
    groups = {}
    for i, (l, c) in enumerate(tree.leaves):
        if l > 0:
            groups.setdefault((l - 1, tuple(x // 2 for x in c)), []).append(i)
    merge = {}
    for par, kids in groups.items():
        if len(kids) != (1 << D) or refine[kids].any():
            continue
        order = sorted(kids, key=lambda i: _octant_of(tree.leaves[i][1], D))
        wpar = restrict(s, w[order])
        Sp = smoothness(s, wpar[None, :], fields)
        if (Sp < 0.5 * s_tilde).all():
            merge[par] = order
    # apply, dropping merges that break the 2:1 balance
    while True:
        leaves = []
        for i, (l, c) in enumerate(tree.leaves):
            if l > 0 and (l - 1, tuple(x // 2 for x in c)) in merge:
                continue
            if refine[i]:
                for off in range(1 << D):
                    leaves.append((l + 1, tuple(2 * c[a] + ((off >> a) & 1) for a in range(D))))
            else:
                leaves.append((l, c))
        leaves += list(merge.keys())
        t = Octree(D, tree.n0, leaves, tree.box)
        bad = t.balance_violations()
        drop = [t.leaves[i] for i in np.nonzero(bad)[0] if t.leaves[i] in merge]
        if not drop:
            break
        for par in drop:
            del merge[par]
    t = t.balanced().morton_sorted()
    # weights of the new leaves
    old = tree.index
    W = np.zeros((len(t.leaves), s.nmodes))
    for i, (l, c) in enumerate(t.leaves):
        if (l, c) in old:
            W[i] = w[old[(l, c)]]
        elif (l, c) in merge:
            W[i] = restrict(s, w[merge[(l, c)]])
        else:
            path, cl, cc = [], l, c          # climb to the old leaf that covers this one
            while (cl, cc) not in old:
                path.append(_octant_of(cc, D))
                cl, cc = cl - 1, tuple(x // 2 for x in cc)
            wv = w[old[(cl, cc)]]
            for o in reversed(path):
                wv = prolong(s, wv, o)
            W[i] = wv
    stats = dict(refined=int(refine.sum()), merged=len(merge), leaves=len(t.leaves))
    return t, W, stats
