"""Pins of the oracle's quadrature and bases against facts fixed by the paper
and by textbook mathematics (no GPU)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import basis as B
from oracle.quadrature import gauss_legendre, tensor_rule

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_legendre_exact_on_monomials(n):
    # an n-point rule integrates x^k exactly for k <= 2n-1 (Sec. 3.5)
    x, w = gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * x ** k).sum() - exact) < 1e-14
    # and not for 2n
    assert abs((w * x ** (2 * n)).sum() - 2.0 / (2 * n + 1)) > 1e-6


def test_gauss_legendre_closed_forms():
    x, w = gauss_legendre(2)
    assert np.allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-16)
    assert np.allclose(w, [1, 1], atol=1e-16)
    x, w = gauss_legendre(3)
    assert np.allclose(x, [-math.sqrt(3 / 5), 0, math.sqrt(3 / 5)], atol=1e-16)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-16)
    x, w = gauss_legendre(4)
    a = math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5))
    b = math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))
    assert np.allclose(x, [-b, -a, a, b], atol=1e-15)
    assert np.allclose(w, [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36,
                           (18 + math.sqrt(30)) / 36, (18 - math.sqrt(30)) / 36], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_legendre_matches_library(n):
    x, w = gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, atol=2e-15) and np.allclose(w, wr, atol=2e-15)


@pytest.mark.parametrize("D,d", [(2, 0), (2, 1), (2, 2), (2, 3), (3, 0), (3, 1), (3, 2), (3, 3)])
def test_legendre_counts_and_orthogonality(D, d):
    # n(d) (Sec. 3.2) and <P_l, P_l'> = delta M_l under the (d+1)-point rule (eq. basis-ortho)
    assert len(B.mode_exponents(D, d)) == B.n_modes(D, d)
    assert B.n_modes(D, d) == (math.comb(d + 2, 2) if D == 2 else math.comb(d + 3, 3))
    xq, wq = tensor_rule(d + 1, D)
    V = B.legendre_values(D, d, xq)
    Mq = (V * wq[:, None]).T @ V
    M = B.legendre_mass(D, d)
    assert np.allclose(Mq, np.diag(M), atol=1e-14 * M.max(), rtol=1e-14)
    # first weight is the cell mean: l_k(1) = 1 normalisation, P_0 = 1
    assert np.allclose(V[:, 0], 1.0)
    assert np.allclose(B.legendre_values(D, d, np.ones((1, D)))[0], 1.0)


def test_legendre_values_against_numpy():
    xi = np.random.default_rng(0).uniform(-1, 1, (50, 3))
    V = B.legendre_values(3, 3, xi)
    G = B.legendre_grads(3, 3, xi)
    for l, e in enumerate(B.mode_exponents(3, 3)):
        c = np.zeros((4, 4, 4))
        c[e] = 1.0
        ref = np.polynomial.legendre.legval3d(xi[:, 0], xi[:, 1], xi[:, 2], c)
        assert np.allclose(V[:, l], ref, atol=1e-14)
        for a in range(3):
            dc = np.polynomial.legendre.legder(c, axis=a)
            dref = np.polynomial.legendre.legval3d(xi[:, 0], xi[:, 1], xi[:, 2], dc)
            assert np.allclose(G[a, :, l], dref, atol=1e-13)


def test_ndiv_table_matches_paper():
    rows = [l.split() for l in open(os.path.join(GOLD, "ndiv_table.txt")) if l.strip() and l[0] != "#"]
    for r in rows:
        D = int(r[0])
        for d, val in enumerate(r[1:]):
            assert B.n_div(D, d) == int(val)
            if D == 3 and d > 3:
                continue  # generator test below covers d <= 3 in 3-D
            basis, _ = B.ldf_basis_exact(D, d)
            assert len(basis) == int(val)


def test_dof_counts_match_paper():
    kv = {l.split()[0]: float(l.split()[1]) for l in open(os.path.join(GOLD, "dof_counts.txt"))
          if l.strip() and l[0] != "#"}
    assert 5 * B.n_modes(3, 1) + B.n_div(3, 1) == kv["N3d_d1"]
    n2 = lambda d: 6 * B.n_modes(2, d) + B.n_div(2, d)  # 5 hydro + B3 Legendre + 2-D LDF
    assert n2(1) == kv["N2d_d1"]
    assert round(n2(1) * 128 ** 2, -4) == kv["NDoF_DG2_128"]
    assert round(n2(1) * 256 ** 2, -5) == kv["NDoF_DG2_256"]
    assert round(n2(2) * 128 ** 2, -4) == kv["NDoF_DG3_128"]


@pytest.mark.parametrize("D,d", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_ldf_basis_divergence_free_orthogonal_graded(D, d):
    basis, norms = B.ldf_basis_exact(D, d)
    for V in basis:
        assert B.ldf_divergence_exact(V) == {}   # exactly divergence-free (App. A)
    for i in range(len(basis)):
        for j in range(i):
            assert B._vinner(list(basis[i]), list(basis[j]), D) == 0  # exactly orthogonal
        assert norms[i] > 0
    degs = B.ldf_degrees(D, d)
    assert degs == sorted(degs) and max(degs) == d
    # span: the count of functions per degree g equals dim V_g^div - dim V_{g-1}^div
    for g in range(d + 1):
        assert degs.count(g) == B.n_div(D, g) - (B.n_div(D, g - 1) if g else 0)
    # float tables reproduce the exact mass under the (d+1)-point rule
    xq, wq = tensor_rule(d + 1, D)
    Phi = B.ldf_values(D, d, xq)
    Mq = np.einsum("cpl,cpm,p->lm", Phi, Phi, wq)
    assert np.allclose(Mq, np.diag(B.ldf_mass(D, d)), atol=1e-13 * Mq.max())
    # pointwise divergence of the float gradient tables vanishes
    dPhi = B.ldf_grads(D, d, xq)
    div = sum(dPhi[a, a] for a in range(D))
    assert np.abs(div).max() < 1e-12


def test_ldf_projection_contamination_matches_paper_table():
    # App. B: projections of u = (a xi1, b xi2) onto the 2-D LDF basis to degree 5
    want = {}
    for line in open(os.path.join(GOLD, "ldf_contamination.txt")):
        if line.strip() and line[0] != "#":
            g, ca, cb = line.split()
            want.setdefault(int(g), []).append((Fraction(ca), Fraction(cb)))
    px = B.ldf_project_exact(2, 5, ({(1, 0, 0): Fraction(1)}, {}))
    py = B.ldf_project_exact(2, 5, ({}, {(0, 1, 0): Fraction(1)}))
    degs = B.ldf_degrees(2, 5)
    got = {}
    for g, a, b in zip(degs, px, py):
        if a != 0 or b != 0:
            got.setdefault(g, []).append((a, b))
    assert sorted(got) == sorted(want)
    for g in want:
        assert sorted(got[g]) == sorted(want[g])
