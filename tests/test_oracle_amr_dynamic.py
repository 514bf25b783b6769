"""Pins of the oracle's dynamic refinement (Sec. 4.4), CPU only:

* smoothness indicator: closed forms for single Legendre modes (S of xi_a is
  2 * 2^D along a and 0 across; S of P_2(xi_a) is 2 int (3 xi)^2 + 8 int 3^2),
  and brute force on random polynomials with finite-difference derivatives
  (stencils exact for the degree) of the oracle's own point evaluation, for
  Legendre variables and for the LDF field;
* prolongation reproduces the parent's polynomial pointwise in every octant;
  restriction after prolongation gives the parent back; restriction of
  arbitrary children is the L2 projection (the residual is orthogonal to
  every parent mode on a fine quadrature) and keeps the mean;
* regrid: refined leaves are exactly those above 2 S~, merged groups are
  below S~/2 as parents, the tree stays 2:1 balanced and tiles the box, mass
  and every conserved total are kept to rounding, the refined cells carry
  the parent's polynomial."""
import numpy as np
import pytest

import workloads as wl
from oracle import amr, dg
from oracle import physics as ph
from oracle.quadrature import tensor_rule

G = 5.0 / 3.0


def _solver(D, d, n0=4, divb=dg.GLM):
    t = amr.Octree.uniform(D, n0)
    return t, dg.DG(t.mesh(), d, divb=divb, glm_ch_fixed=3.0)


@pytest.mark.parametrize("D", [2, 3])
def test_smoothness_closed_forms(D):
    t, s = _solver(D, 3)
    exps = [tuple(e) for e in __import__("oracle.basis", fromlist=["x"]).mode_exponents(D, 3)]
    for a in range(D):
        e1 = tuple(1 if b == a else 0 for b in range(D))
        e2 = tuple(2 if b == a else 0 for b in range(D))
        w = np.zeros((2, s.nmodes))
        w[0, exps.index(e1)] = 1.0          # rho = xi_a
        w[1, exps.index(e2)] = 1.0          # rho = P_2(xi_a)
        S = amr.smoothness(s, w, fields=(ph.RHO,))[:, 0, :]
        vol = 2.0 ** D
        assert np.isclose(S[0, a], 2.0 * vol, rtol=1e-13)
        assert np.isclose(S[1, a], 2.0 * 9.0 * (2.0 / 3.0) * vol / 2.0 + 8.0 * 9.0 * vol, rtol=1e-13)
        for b in range(D):
            if b != a:
                assert abs(S[0, b]) < 1e-13 and abs(S[1, b]) < 1e-13


def _fd(fun, x, a, k, h=1e-2):
    e = np.zeros(x.shape[1])
    e[a] = h
    f = {j: fun(x + j * e) for j in (-2, -1, 0, 1, 2)}
    if k == 1:
        return (-f[2] + 8 * f[1] - 8 * f[-1] + f[-2]) / (12 * h)
    if k == 2:
        return (-f[2] + 16 * f[1] - 30 * f[0] + 16 * f[-1] - f[-2]) / (12 * h * h)
    return (f[2] - 2 * f[1] + 2 * f[-1] - f[-2]) / (2 * h ** 3)


@pytest.mark.parametrize("D,d,divb", [(2, 3, dg.GLM), (3, 2, dg.GLM), (3, 3, dg.POWELL), (2, 2, dg.POWELL)])
def test_smoothness_brute_force(D, d, divb):
    t, s = _solver(D, d, divb=divb)
    rng = np.random.default_rng(10 * D + d)
    w = rng.normal(size=(3, s.nmodes))
    fields = (ph.RHO, ph.B1, ph.B2)
    S = amr.smoothness(s, w, fields=fields)
    xq, wq = tensor_rule(d + 3, D)
    for c in range(3):
        for i, v in enumerate(fields):
            fun = lambda x, c=c, v=v: s.nodal(w[c:c + 1], xi=x)[v, 0]
            for a in range(D):
                ref = sum(2.0 ** (2 * k - 1) * (_fd(fun, xq, a, k) ** 2 * wq).sum() for k in range(1, d + 1))
                assert np.isclose(S[c, i, a], ref, rtol=1e-6, atol=1e-9), (c, v, a, S[c, i, a], ref)


@pytest.mark.parametrize("D,d,divb", [(2, 2, dg.GLM), (3, 3, dg.GLM), (3, 2, dg.POWELL), (2, 3, dg.POWELL)])
def test_prolongation_and_restriction(D, d, divb):
    t, s = _solver(D, d, divb=divb)
    rng = np.random.default_rng(5 + d)
    wp = rng.normal(size=s.nmodes)
    kids = np.stack([amr.prolong(s, wp, o) for o in range(1 << D)])
    xr = rng.uniform(-1, 1, (20, D))
    for o in range(1 << D):
        sh = np.array([2 * ((o >> a) & 1) - 1 for a in range(D)], dtype=float)
        uc = s.nodal(kids[o][None], xi=xr)
        up = s.nodal(wp[None], xi=0.5 * (xr + sh))
        assert np.allclose(uc, up, rtol=0, atol=1e-12 * np.abs(up).max())
    assert np.allclose(amr.restrict(s, kids), wp, rtol=0, atol=1e-12 * np.abs(wp).max())
    # arbitrary children: L2 projection (residual orthogonal to the parent's modes) and the mean kept
    wc = rng.normal(size=(1 << D, s.nmodes))
    wr = amr.restrict(s, wc)
    xf, wf = tensor_rule(d + 2, D)
    tabs = s._basis_at(xf)
    resid = np.zeros(s.nmodes)
    for o in range(1 << D):
        sh = np.array([2 * ((o >> a) & 1) - 1 for a in range(D)], dtype=float)
        xp = 0.5 * (xf + sh)
        diff = s.nodal(wc[o][None], xi=xf) - s.nodal(wr[None], xi=xp)
        resid += s.project_test(diff, s._basis_at(xp), wf * 2.0 ** -D)[0]
    assert np.abs(resid).max() < 1e-12 * np.abs(wc).max()
    mk = s.cell_means(wc).mean(axis=1)
    assert np.allclose(s.cell_means(wr[None])[:, 0], mk, rtol=0, atol=1e-13)


@pytest.mark.parametrize("divb", [dg.GLM, dg.POWELL])
def test_regrid_orszag_tang(divb):
    D, d = 2, 2
    t = amr.Octree.uniform(D, 8)
    s = dg.DG(t.mesh(), d, divb=divb, glm_ch_fixed=3.0)
    w = s.project(dg.conserved_field(wl.OrszagTang(), G, s.nvar))
    S = amr.smoothness(s, w)
    s_tilde = float(np.quantile(S.max(axis=(1, 2)), 0.8)) / 2.0
    t2, w2, st = amr.regrid(t, s, w, s_tilde=s_tilde)
    assert st["refined"] == int((S > 2 * s_tilde).any(axis=(1, 2)).sum()) > 0
    assert not t2.balance_violations().any()
    s2 = dg.DG(t2.mesh(), d, divb=divb, glm_ch_fixed=3.0)
    vol1 = s.mesh.h ** D
    vol2 = s2.mesh.h ** D
    tot1 = (s.cell_means(w) * vol1).sum(axis=1)
    tot2 = (s2.cell_means(w2) * vol2).sum(axis=1)
    assert np.allclose(tot1, tot2, rtol=0, atol=1e-13 * np.abs(tot1).max())
    assert np.isclose(vol2.sum(), 1.0, rtol=1e-14)
    # refined cells carry the parent's polynomial
    rng = np.random.default_rng(1)
    xr = rng.uniform(-1, 1, (10, D))
    for i, (l, c) in enumerate(t2.leaves):
        if l == 1:
            p = t.index[(0, tuple(x // 2 for x in c))]
            sh = np.array([2 * (x & 1) - 1 for x in c], dtype=float)
            assert np.allclose(s2.nodal(w2[i][None], xi=xr), s.nodal(w[p][None], xi=0.5 * (xr + sh)), atol=1e-12)
    # a second regrid with a large threshold merges the refined groups back
    t3, w3, st3 = amr.regrid(t2, s2, w2, s_tilde=1e9)
    assert st3["merged"] == st["refined"] and len(t3.leaves) == len(t.leaves)
    back = {lf: i for i, lf in enumerate(t3.leaves)}
    for i, lf in enumerate(t.leaves):
        assert np.allclose(w3[back[lf]], w[i], atol=1e-12 * np.abs(w).max())


@pytest.mark.parametrize("D", [2, 3])
def test_balance_refines_the_coarse_side_only(D):
    """A cell refined twice inside a uniform level-0 grid: the leaves next to
    its level-2 children get refined once, the level-2 leaves are left as
    they are, and the result has no face neighbours two levels apart."""
    t = amr.Octree.uniform(D, 4)
    t = t.refine(np.array([c == (1,) * D for _, c in t.leaves]))
    t = t.refine(np.array([l == 1 and c == (2,) * D for l, c in t.leaves]))
    deep = {lf for lf in t.leaves if lf[0] == 2}
    bad = t.balance_violations()
    assert all(t.leaves[i][0] == 0 for i in np.nonzero(bad)[0])      # only coarse leaves are flagged
    tb = t.balanced()
    assert max(l for l, _ in tb.leaves) == 2 and deep <= set(tb.leaves)
    assert not tb.balance_violations().any()
    tb.mesh()                                                        # builds (raises on a 2:1 violation)
