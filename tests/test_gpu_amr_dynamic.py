"""GPU parity of the dynamic refinement (Sec. 4.4) against the oracle:
smoothness indicators of leaves, the regrid decision (refined leaves, merged
sibling groups, 2:1 balance, Morton order as sets of leaves), the transferred
weights (copy, prolongation through every level, restriction) and steps on
the regridded mesh.  Thresholds are taken away from every indicator by a
relative margin, so that no decision rests on rounding."""
import sys
import warnings

import numpy as np
import pytest

import workloads as wl
from oracle import amr, dg
from oracle import physics as ph
from parity_util import rel_l1, to_cells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
G = 5.0 / 3.0
RHO_B = (ph.RHO, ph.B1, ph.B2, ph.B3)


def _announce(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


def _bump(D, width=0.08):
    """A Gaussian density bump at (0.4, 0.55[, 0.5]) on a uniform background:
    large indicators near it, none far away (numpy evaluation only)."""
    c = np.array([0.4, 0.55, 0.5])[:D]

    def f(x):
        r2 = ((x - c) ** 2).sum(axis=1)
        one = np.ones(x.shape[0])
        b = 1.0 / np.sqrt(4 * np.pi)
        return dict(rho=1.0 + 0.5 * np.exp(-r2 / (2 * width ** 2)), v=[0 * one, 0 * one, 0 * one], p=one,
                    B=[b * one, 0.5 * b * one, 0 * one], psi=0 * one)
    return f


def _pair(tree, d, field, ch=3.0):
    from paper_1806_02343_amd import DG
    octree = None if all(l == 0 for l, _ in tree.leaves) else (tree.levels(), tree.coords())
    if octree is None:
        gpu = DG(tree.D, d, tree.n0, glm_ch_fixed=ch)
        orc_tree = tree
    else:
        gpu = DG(tree.D, d, tree.n0, glm_ch_fixed=ch, octree=octree)
        orc_tree = tree
    orc = dg.DG(orc_tree.mesh(), d, glm_ch_fixed=ch)
    wo = orc.project(dg.conserved_field(field, G, 9))
    wg = torch.as_tensor(orc.to_abi(wo, gpu.ld), device="cuda")
    return gpu, wg, orc, wo


def _uniform_tree(D, n0):
    # the oracle's uniform leaves in the library's cell order (index i + n0 (j + n1 k))
    t = amr.Octree.uniform(D, n0)
    return t


def _safe_threshold(orc, tree, wo, q):
    """A threshold S~ near the q-quantile of the leaves' indicators with every
    leaf indicator at least 1e-6 (relative) away from 2 S~ and every complete
    group's parent indicator away from S~/2."""
    S = amr.smoothness(orc, wo, RHO_B).max(axis=(1, 2))
    groups = {}
    for i, (l, c) in enumerate(tree.leaves):
        if l > 0:
            groups.setdefault((l - 1, tuple(x // 2 for x in c)), []).append(i)
    Sp = []
    for kids in groups.values():
        if len(kids) == 1 << tree.D:
            kids = sorted(kids, key=lambda i: amr._octant_of(tree.leaves[i][1], tree.D))
            Sp.append(amr.smoothness(orc, amr.restrict(orc, wo[kids])[None], RHO_B).max())
    Sp = np.array(Sp)
    # thresholds in the gaps between distinct indicator values (symmetric
    # states repeat values), starting at the q-quantile
    ss = np.sort(S)
    u = ss[np.concatenate([[True], np.diff(ss) > 1e-9 * ss.max()])]
    k0 = min(int(np.searchsorted(u, np.quantile(S, q))), len(u) - 2)
    for k in list(range(k0, len(u) - 1)) + list(range(k0 - 1, -1, -1)):
        if u[k + 1] <= u[k] * (1 + 1e-5):
            continue
        st = 0.25 * (u[k] + u[k + 1])
        if np.all(np.abs(S / (2 * st) - 1) > 1e-6) and (Sp.size == 0 or np.all(np.abs(Sp / (0.5 * st) - 1) > 1e-6)):
            return st, S, Sp
    raise RuntimeError("no safe threshold")


def _check_regrid(gpu, wg, orc, wo, tree, s_tilde, max_level, d, ch=3.0):
    t2, W2, st = amr.regrid(tree, orc, wo, s_tilde=s_tilde, fields=RHO_B, max_level=max_level)
    new, wn = gpu.regrid(wg, s_tilde=s_tilde, max_level=max_level, glm_ch_fixed=ch)
    keys_g = [(int(l), tuple(int(x) for x in c[:tree.D])) for l, c in zip(new.level, new.ijk)]
    assert sorted(keys_g) == sorted(t2.leaves)
    assert keys_g == t2.leaves                       # same Morton order
    Wg = to_cells(wn, len(keys_g))
    scale = np.abs(W2).max()
    assert np.abs(Wg - W2).max() < 1e-12 * scale
    return t2, W2, st, new, wn


@pytest.mark.parametrize("D,d,n0,field", [(2, 2, 16, "ot"), (2, 3, 12, "ot"), (3, 2, 6, "smooth"), (3, 1, 8, "smooth")])
def test_indicator_matches_oracle(D, d, n0, field):
    _announce("amr indicator", D, d, n0)
    f = wl.OrszagTang() if field == "ot" else wl.Smooth(31, 3)
    tree = _uniform_tree(D, n0)
    gpu, wg, orc, wo = _pair(tree, d, f)
    from paper_1806_02343_amd.binding import AMR_FIELDS_RHO_B
    for mask, fields in ((AMR_FIELDS_RHO_B, RHO_B), (0x1FF, tuple(range(9))), (1 << 4, (ph.EN,))):
        S = gpu.amr_indicator(wg, mask).cpu().numpy()
        So = amr.smoothness(orc, wo, fields).max(axis=(1, 2))
        assert np.abs(S - So).max() <= 1e-12 * So.max(), (mask, np.abs(S - So).max() / So.max())


@pytest.mark.parametrize("D,d,n0", [(2, 2, 16), (2, 1, 16), (3, 2, 6)])
def test_regrid_from_uniform_matches_oracle_and_steps(D, d, n0):
    _announce("amr regrid uniform", D, d, n0)
    f = wl.OrszagTang() if D == 2 else wl.Smooth(31, 3)
    tree = _uniform_tree(D, n0)
    gpu, wg, orc, wo = _pair(tree, d, f)
    s_tilde, S, _ = _safe_threshold(orc, tree, wo, 0.8)
    # the steps' fixed c_h above twice the largest signal speed (about 4.4 on
    # the Orszag-Tang state), so the runtime c_h check passes
    chs = 5.0 if D == 2 else 3.0
    t2, W2, st, new, wn = _check_regrid(gpu, wg, orc, wo, tree, s_tilde, 3, d, ch=chs)
    assert st["refined"] > 0 and len(t2.leaves) > len(tree.leaves)
    # two SSP-RK3 steps on the regridded mesh
    orc2 = dg.DG(t2.mesh(), d, glm_ch_fixed=chs)
    w2 = W2.copy()
    for _ in range(2):
        w2, dt, ch, k = orc2.step(w2)
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        new.step(wn, 2)
    err = rel_l1(orc2, to_cells(wn, len(t2.leaves)), w2, ch=chs)
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("D,d", [(2, 2), (3, 1), (3, 3)])
def test_regrid_with_merges_matches_oracle(D, d):
    """From a refined tree: groups in smooth regions merge, leaves at the
    features split (possibly two levels below a merge, with balance
    refinements), and a second regrid runs on the result."""
    _announce("amr regrid merges", D, d)
    n0 = 8 if D == 2 else 4
    tree = amr.Octree.uniform(D, n0)
    tree = tree.refine(np.ones(len(tree.leaves), dtype=bool)).morton_sorted()   # everything at level 1
    gpu, wg, orc, wo = _pair(tree, d, _bump(D))
    s_tilde, S, Sp = _safe_threshold(orc, tree, wo, 0.9)
    t2, W2, st, new, wn = _check_regrid(gpu, wg, orc, wo, tree, s_tilde, 3, d)
    assert st["merged"] > 0 and st["refined"] > 0, st
    assert not t2.balance_violations().any()
    # totals kept
    orc2 = dg.DG(t2.mesh(), d, glm_ch_fixed=3.0)
    tot1 = (orc.cell_means(wo) * orc.mesh.h ** D).sum(axis=1)
    tot2 = (orc2.cell_means(to_cells(wn, len(t2.leaves))) * orc2.mesh.h ** D).sum(axis=1)
    assert np.allclose(tot1, tot2, rtol=0, atol=1e-13 * np.abs(tot1).max())
    # a second regrid from the GPU state on the new handle
    s2, _, _ = _safe_threshold(orc2, t2, W2, 0.5)
    _check_regrid(new, wn, orc2, W2, t2, s2, 3, d)


def test_regrid_errors():
    from paper_1806_02343_amd import DG, DGError
    from paper_1806_02343_amd.binding import DG_EINVAL, DG_EUNSUPPORTED
    _announce("amr errors")
    gp = DG(3, 2, 4, divb=dg.POWELL)
    wp = gp.empty_state()
    with pytest.raises(DGError) as e:
        gp.amr_indicator(wp)
    assert e.value.code == DG_EUNSUPPORTED
    g = DG(2, 2, 8, glm_ch_fixed=3.0)
    w = g.empty_state()
    g.project_field(wl.OrszagTang(), w)
    with pytest.raises(DGError) as e:
        g.regrid(w, s_tilde=-1.0, glm_ch_fixed=3.0)
    assert e.value.code == DG_EINVAL
    # a handle whose leaves are not the plan's
    other = DG(2, 2, 8, glm_ch_fixed=3.0)
    n, _ = None, None
    import ctypes
    nn = ctypes.c_int64()
    g._check(g.lib.dg_amr_plan(g.h, ctypes.c_void_p(w.data_ptr()), 0xE1, 1e-3, 2, ctypes.byref(nn)))
    rc = g.lib.dg_amr_transfer(g.h, ctypes.c_void_p(w.data_ptr()), other.h, ctypes.c_void_p(other.empty_state().data_ptr()))
    assert rc == DG_EINVAL
