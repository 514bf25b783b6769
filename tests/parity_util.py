"""Shared helpers of the GPU parity tests: build an oracle scheme and a HIP
handle for the same configuration and seeded input, and compare them."""
import numpy as np

import workloads as wl
from oracle import dg
from oracle.quadrature import tensor_rule

G = 5.0 / 3.0


def make_pair(D, d, n, divb=0, precision=0, box=1.0, field=None, limiter=0, cfl=0.3, **kw):
    import torch
    from paper_1806_02343_amd import DG
    field = field if field is not None else wl.Smooth(1000 * D + d, D)
    gpu = DG(D, d, n, box=box, divb=divb, precision=precision, limiter=limiter, cfl=cfl, **kw)
    wg = gpu.empty_state()
    gpu.project_field(field, wg)
    torch.cuda.synchronize()
    orc = dg.DG(dg.Mesh.uniform(D, n, box), d, divb=divb, cfl=cfl)
    wo = orc.project(dg.conserved_field(field, G, orc.nvar))
    return gpu, wg, orc, wo


def to_cells(t, ncells):
    """[nmodes][ld] device tensor -> oracle layout [cell][mode] (float64 numpy)."""
    return t[:, :ncells].double().cpu().numpy().T.copy()


def rel_l1(orc, w_test, w_ref, ch=1.0):
    """Per-variable relative L1 error of nodal values at (d+3)^D points
    (eq. lp_norm); psi is measured against c_h ||B||_1."""
    xq, wq = tensor_rule(orc.d + 3, orc.D)
    tabs = orc._basis_at(xq)
    Ut = orc.nodal(w_test, tabs=tabs)
    Ur = orc.nodal(w_ref, tabs=tabs)
    err = (np.abs(Ut - Ur) * wq).sum(axis=(1, 2))
    ref = (np.abs(Ur) * wq).sum(axis=(1, 2))
    out = err / np.maximum(ref, 1e-300)
    if orc.nvar == 9:
        bn = ref[5:8].sum()
        out[8] = err[8] / max(ch * bn, 1e-300)
    return out


def block_rel_max(a, b, orc, floor=1e-3):
    """max |a-b| / max |b| per variable block (modal arrays [cell][mode]).
    The denominator is floored at `floor` x the largest block maximum, so a
    block that is zero in exact arithmetic (e.g. momentum of a state at rest)
    is judged against the state's scale instead of its own rounding noise."""
    res = []
    n = orc.n
    gmax = max(np.abs(b).max(), 1e-300)
    for j in range(len(orc.leg_vars)):
        sl = slice(j * n, (j + 1) * n)
        res.append(np.abs(a[:, sl] - b[:, sl]).max() / max(np.abs(b[:, sl]).max(), floor * gmax))
    if orc.nldf:
        sl = slice(len(orc.leg_vars) * n, None)
        res.append(np.abs(a[:, sl] - b[:, sl]).max() / max(np.abs(b[:, sl]).max(), floor * gmax))
    return np.array(res)


class LeafIndex:
    """Lookup of octree leaves (level, integer coordinates on the level grid
    of n0 2^level cells per periodic axis) by sorted integer keys, for leaf
    sets too large for a Python dictionary of tuples."""

    def __init__(self, level, ijk, n0, D=3):
        self.n0, self.D = n0, D
        self.level = np.asarray(level, dtype=np.int64)
        self.ijk = np.asarray(ijk, dtype=np.int64)[:, :D]
        self.lmax = int(self.level.max()) if len(self.level) else 0
        keys = self._keys(self.level, self.ijk)
        self.order = np.argsort(keys, kind="stable")
        self.sorted = keys[self.order]

    def _keys(self, level, ijk):
        m = self.n0 << self.lmax
        k = level.astype(np.int64)
        for a in range(self.D):
            k = k * m + ijk[..., a]
        return k

    def find(self, level, c):
        """Index of leaf (level, c) (c wrapped periodically), or -1."""
        if level < 0 or level > self.lmax:
            return -1
        m = self.n0 << level
        c = np.array([x % m for x in c], dtype=np.int64)
        key = self._keys(np.int64(level), c[None, :])[0]
        p = np.searchsorted(self.sorted, key)
        return int(self.order[p]) if p < len(self.sorted) and self.sorted[p] == key else -1

    def local_mesh(self, i):
        """The leaf i, its face neighbours and every face touching leaf i, as
        an oracle Mesh (leaf i is cell 0) in the oracle octree's face
        conventions (a face listed from its left cell's +e_a side; a coarse
        side on quarter q, bit t of q set for the upper half of the t-th
        tangential axis), plus the global indices of the mesh's cells.  The
        oracle's right-hand side of cell 0 on this mesh is that of leaf i on
        the whole octree."""
        D = self.D
        l = int(self.level[i])
        c = [int(x) for x in self.ijk[i]]
        cells = [i]

        def cid(j):
            assert j >= 0, "mesh is not complete or not 2:1 balanced"
            if j not in cells:
                cells.append(j)
            return cells.index(j)

        faces = []
        for a in range(D):
            tang = [b for b in range(D) if b != a]
            qc = sum(((c[b] & 1) << k) for k, b in enumerate(tang))
            F = []
            # +a side
            nc = list(c)
            nc[a] += 1
            j = self.find(l, nc)
            if j >= 0:
                F.append((0, cid(j), -1, -1))
            elif l > 0 and self.find(l - 1, [x // 2 for x in nc]) >= 0:
                F.append((0, cid(self.find(l - 1, [x // 2 for x in nc])), -1, qc))
            else:
                for q in range(1 << (D - 1)):
                    ch = [2 * x for x in nc]
                    for k, b in enumerate(tang):
                        ch[b] += (q >> k) & 1
                    F.append((0, cid(self.find(l + 1, ch)), q, -1))
            # -a side
            nc = list(c)
            nc[a] -= 1
            j = self.find(l, nc)
            if j >= 0:
                F.append((cid(j), 0, -1, -1))
            elif l > 0 and self.find(l - 1, [x // 2 for x in nc]) >= 0:
                F.append((cid(self.find(l - 1, [x // 2 for x in nc])), 0, qc, -1))
            else:
                for q in range(1 << (D - 1)):
                    ch = [2 * x for x in nc]
                    ch[a] += 1
                    for k, b in enumerate(tang):
                        ch[b] += (q >> k) & 1
                    F.append((cid(self.find(l + 1, ch)), 0, -1, q))
            F = np.array(F, dtype=np.int64)
            faces.append(dict(axis=a, L=F[:, 0], R=F[:, 1], subL=F[:, 2], subR=F[:, 3]))
        lv = self.level[cells]
        h = 1.0 / (self.n0 * (2.0 ** lv))
        centers = (self.ijk[cells] + 0.5) * h[:, None]
        return dg.Mesh(D, h, centers, faces), np.array(cells)

    def region_mesh(self, i, layers):
        """Oracle mesh of the leaves within `layers` face layers of leaf i, with
        every face touching the inner layers (leaf i is cell 0), and the global
        leaf indices of its cells.  The scheme's value at leaf i after `layers`
        stages is exact on it: a stage needs one face layer."""
        shells = [[i]]
        seen = {i}
        for _ in range(layers):
            nxt = []
            for x in shells[-1]:
                _, cells = self.local_mesh(x)
                for y in cells.tolist():
                    if y not in seen:
                        seen.add(y)
                        nxt.append(y)
            shells.append(nxt)
        order = [x for sh in shells for x in sh]
        pos = {x: k for k, x in enumerate(order)}
        faces = [set() for _ in range(self.D)]
        for x in [x for sh in shells[:-1] for x in sh]:
            m, cells = self.local_mesh(x)
            for f in m.faces:
                for L, R, sL, sR in zip(f["L"], f["R"], f["subL"], f["subR"]):
                    faces[f["axis"]].add((pos[int(cells[L])], pos[int(cells[R])], int(sL), int(sR)))
        fl = []
        for a in range(self.D):
            F = np.array(sorted(faces[a]), dtype=np.int64)
            fl.append(dict(axis=a, L=F[:, 0], R=F[:, 1], subL=F[:, 2], subR=F[:, 3]))
        lv = self.level[order]
        h = 1.0 / (self.n0 * (2.0 ** lv))
        return dg.Mesh(self.D, h, (self.ijk[order] + 0.5) * h[:, None], fl), np.array(order)
