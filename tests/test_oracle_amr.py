"""Pins of the oracle's octree AMR (no GPU): a uniform octree reproduces the
uniform grid, hanging faces keep the scheme conservative and free-stream
preserving, coarse traces at sub-face points equal fine traces for fields
the basis represents exactly, and the advected density peaks (an exact
entropy wave) converge with the degree."""
import numpy as np
import pytest

import workloads as wl
from oracle import dg
from oracle.amr import Octree
from oracle.quadrature import tensor_rule

G = 5.0 / 3.0


def small_tree(D, n0=4, seed=0):
    """n0^D base grid with a refined 2x..x2 block and one doubly refined cell."""
    t = Octree.uniform(D, n0)
    flags = np.array([all(1 <= c[a] <= 2 for a in range(D)) for _, c in t.leaves])
    t = t.refine(flags)
    flags = np.array([l == 1 and all(c[a] == 3 for a in range(D)) for l, c in t.leaves])
    t = t.refine(flags).balanced()
    return t.morton_sorted()


def test_uniform_octree_equals_uniform_grid():
    t = Octree.uniform(3, 3)
    m1, m2 = t.mesh(), dg.Mesh.uniform(3, 3)
    s1, s2 = dg.DG(m1, 2), dg.DG(m2, 2)
    w = s2.project(dg.conserved_field(wl.Smooth(5, 3), G, 9))
    assert np.allclose(s1.rhs(w, 1.3, 0.2), s2.rhs(w, 1.3, 0.2), rtol=0, atol=1e-13 * np.abs(s2.rhs(w, 1.3, 0.2)).max())


@pytest.mark.parametrize("D", [2, 3])
def test_tree_is_balanced_and_has_hanging_faces(D):
    t = small_tree(D)
    assert not t.balance_violations().any()
    m = t.mesh()
    nh = sum(int((f["subL"] >= 0).sum() + (f["subR"] >= 0).sum()) for f in m.faces)
    assert nh > 0
    # every cell side is covered: full faces count 1, quarter faces 1/2^(D-1)
    cover = np.zeros((m.ncells, D, 2))
    for f in m.faces:
        a = f["axis"]
        for L, R, sl, sr in zip(f["L"], f["R"], f["subL"], f["subR"]):
            cover[L, a, 1] += 1.0 if sl < 0 else 0.5 ** (D - 1)
            cover[R, a, 0] += 1.0 if sr < 0 else 0.5 ** (D - 1)
    assert np.allclose(cover, 1.0)


@pytest.mark.parametrize("D,d", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_free_stream_and_conservation_on_amr(D, d):
    t = small_tree(D)
    m = t.mesh()
    s = dg.DG(m, d, glm_ch_fixed=3.0)
    u = np.array([1.3, 0.2, -0.1, 0.3, 4.0, 0.7, -0.4, 0.5, 0.0])
    w = s.project(lambda x: np.tile(u[:, None], (1, x.shape[0])))
    r = s.rhs(w, 3.0, 0.0)
    assert np.abs(r).max() < 1e-12 * (2.0 / m.h.min()) * 10
    w = s.project(dg.conserved_field(wl.Smooth(7, D), G, 9))
    vol = m.h ** D
    tot0 = (w[:, ::s.n] * vol[:, None]).sum(0)
    for _ in range(2):
        w, dt, ch, k = s.step(w)
    tot1 = (w[:, ::s.n] * vol[:, None]).sum(0)
    assert np.all(np.abs(tot1 - tot0)[:8] < 1e-14 * np.maximum(np.abs(w[:, ::s.n]).max(0)[:8], 1.0))


def test_subface_traces_match_for_polynomial_field():
    # a global polynomial of degree <= d is represented exactly on every cell,
    # so the coarse trace at the sub-face points equals the fine trace there
    t = small_tree(3)
    m = t.mesh()
    d = 2
    s = dg.DG(m, d)
    poly = lambda x: 1.0 + 0.3 * x[:, 0] - 0.2 * x[:, 1] ** 2 + 0.5 * x[:, 0] * x[:, 2]
    field = lambda x: np.stack([poly(x)] * 9)
    w = s.project(field)
    checked = 0
    for f in m.faces:
        a = f["axis"]
        for L, R, sl, sr in zip(f["L"], f["R"], f["subL"], f["subR"]):
            if sl < 0 and sr < 0:
                continue
            xl = s.face_points(a, +1, sl)
            xr = s.face_points(a, -1, sr)
            ul = s.nodal(w[[L]], xi=xl)[0, 0]
            ur = s.nodal(w[[R]], xi=xr)[0, 0]
            # only faces away from the periodic wrap (the polynomial is not periodic)
            pl = m.centers[L] + 0.5 * m.h[L] * xl
            pr = m.centers[R] + 0.5 * m.h[R] * xr
            if np.abs(pl - pr).max() > 1e-12:
                continue
            assert np.allclose(ul, ur, atol=1e-13)
            assert np.allclose(ul, poly(pl), atol=1e-13)
            checked += 1
    assert checked > 0


def test_advected_peaks_entropy_wave_converges_with_degree():
    # Gaussian peaks in a uniform flow with uniform p and B: exact entropy wave
    pk = wl.Peaks(3000, npk=2, width=0.12)
    t = Octree.uniform(3, 4)
    flags = pk.refine_flags(np.array([[(c[a] + 0.5) / 4 for a in range(3)] for _, c in t.leaves]), 0.3)
    t = t.refine(flags).balanced().morton_sorted()
    m = t.mesh()
    errs = []
    for d in (1, 2):
        s = dg.DG(m, d, glm_ch_fixed=2.5)
        w = s.project(dg.conserved_field(pk, G, 9))
        tt = 0.0
        for _ in range(3):
            w, dt, ch, k = s.step(w)
            tt += dt
        xq, wq = tensor_rule(d + 3, 3)
        U = s.nodal(w, xi=xq)
        x = m.centers[:, None, :] + 0.5 * m.h[:, None, None] * xq[None]
        ex = pk(x.reshape(-1, 3), t=tt)["rho"].reshape(m.ncells, -1)
        errs.append((np.abs(U[0] - ex) * wq * (m.h ** 3)[:, None] / 8).sum())
    assert errs[1] < 0.7 * errs[0], errs


def test_local_mesh_gives_the_whole_octree_rhs():
    """The full-size octree parity samples leaves and runs the oracle on each
    leaf's local mesh (the leaf, its face neighbours and the faces touching
    it).  On the peaks recipe's octree over an 8^3 base grid that local
    right-hand side equals the whole mesh's for leaves on every kind of face
    (same level, coarse and fine sides of hanging faces, periodic wrap)."""
    from parity_util import LeafIndex
    pk = wl.Peaks(3000, npk=3, width=0.08)
    lv, ijk = wl.peaks_leaves(pk, n0=8, r1=0.25, r2=0.15)
    t = Octree.from_arrays(3, 8, lv, ijk)
    orc = dg.DG(t.mesh(), 1, glm_ch_fixed=3.5)
    wo = orc.project(dg.conserved_field(pk, G, 9))
    R = orc.rhs(wo, 3.5, 1.5)
    idx = LeafIndex(lv, ijk, 8)
    rng = np.random.default_rng(5)
    picks = set(rng.choice(len(lv), 12, replace=False).tolist())
    for l in (0, 1, 2):  # leaves next to a level change, of each level
        cand = np.flatnonzero(lv == l)
        for i in rng.permutation(cand):
            m, cells = idx.local_mesh(int(i))
            if len(np.unique(idx.level[cells])) > 1:
                picks.add(int(i))
                break
    picks.add(int(np.flatnonzero((ijk[:, :3] == 0).all(axis=1))[0]))  # the origin's corner leaf
    kinds = set()
    for i in sorted(picks):
        m, cells = idx.local_mesh(i)
        for f in m.faces:
            kinds |= {("coarse left" if s >= 0 else "full") for s in f["subL"]}
            kinds |= {("coarse right" if s >= 0 else "full") for s in f["subR"]}
        loc = dg.DG(m, 1, glm_ch_fixed=3.5).rhs(wo[cells], 3.5, 1.5)[0]
        scale = np.abs(R[i]).max()
        assert np.abs(loc - R[i]).max() <= 1e-13 * scale, (i, np.abs(loc - R[i]).max(), scale)
    assert kinds == {"full", "coarse left", "coarse right"}


def test_region_mesh_gives_the_whole_octree_step():
    """The full-size octree step parity runs the oracle on the leaves within
    three face layers of a sampled leaf (every face touching the inner two
    layers).  On the peaks recipe's small octree one SSP-RK3 step on that
    region equals the whole mesh's step at the leaf; two layers do not."""
    from parity_util import LeafIndex
    pk = wl.Peaks(3000, npk=3, width=0.08)
    lv, ijk = wl.peaks_leaves(pk, n0=8, r1=0.25, r2=0.15)
    orc = dg.DG(Octree.from_arrays(3, 8, lv, ijk).mesh(), 1, glm_ch_fixed=3.5)
    wo = orc.project(dg.conserved_field(pk, G, 9))

    def step(o, w, dt=1e-3, ch=3.5, kappa=1.5):
        u1 = w + dt * o.rhs(w, ch, kappa)
        u2 = 0.75 * w + 0.25 * (u1 + dt * o.rhs(u1, ch, kappa))
        return w / 3.0 + 2.0 / 3.0 * (u2 + dt * o.rhs(u2, ch, kappa))

    full = step(orc, wo)
    idx = LeafIndex(lv, ijk, 8)
    rng = np.random.default_rng(3)
    short = 0.0
    for i in rng.choice(len(lv), 8, replace=False):
        scale = np.abs(full[i]).max()
        m, cells = idx.region_mesh(int(i), 3)
        assert np.abs(step(dg.DG(m, 1, glm_ch_fixed=3.5), wo[cells])[0] - full[i]).max() <= 1e-14 * scale
        m, cells = idx.region_mesh(int(i), 2)
        short = max(short, np.abs(step(dg.DG(m, 1, glm_ch_fixed=3.5), wo[cells])[0] - full[i]).max() / scale)
    assert short > 1e-6
