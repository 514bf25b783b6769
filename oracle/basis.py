"""Modal bases of the DG scheme (oracle; test infrastructure only).

Legendre basis (Sec. 3.2, eq. legendre-3d): P_{k1k2k3}(xi) = l_k1(xi1) l_k2(xi2)
l_k3(xi3) with k1+k2+k3 <= d, l_k the univariate Legendre polynomial with the
standard normalisation l_k(1) = 1, so the first weight is the cell mean and
the mass diagonal is M = prod_i 2/(2k_i+1) (orthogonality, eq. basis-ortho).
Modes are indexed by total degree first, then k1 descending, then k2
descending (the paper leaves the single-integer labelling open).

Locally divergence-free (LDF) basis (Sec. 3.3, App. A "Generation of basis
functions"): curls of a pool of vector polynomials of degree <= d+1, zero
curls dropped, stably sorted by total degree, then Gram-Schmidt
orthogonalised under the L2 inner product of the magnetic components until
N_div = D n(d) - n(d-1) (eq. dimVdiv) vectors are collected.  Pool: the
Legendre products of degree <= d+1 in the order above, placed first in the x,
then the y, then the z component.  In 2-D the divergence-free pair (B1, B2)
comes from curls of (0, 0, Q).  All of it is done in exact rational
arithmetic; no normalisation and no sign change is applied.
"""
from fractions import Fraction
from functools import lru_cache
import itertools

import numpy as np

# --------------------------------------------------------------------------
# counting (Sec. 3.2, App. A)


def n_modes(D, d):
    """n(d): dimension of the scalar polynomials of total degree <= d in D variables."""
    if d < 0:
        return 0
    if D == 2:
        return (d + 1) * (d + 2) // 2
    if D == 3:
        return (d + 1) * (d + 2) * (d + 3) // 6
    raise ValueError(D)


def n_div(D, d):
    """N_div = D n(d) - n(d-1)  (eq. dimVdiv, Table tab:ndiv)."""
    return D * n_modes(D, d) - n_modes(D, d - 1)


def mode_exponents(D, d):
    """List of exponent tuples (k1,..,kD), graded by total degree, then k1
    descending, then k2 descending."""
    out = []
    for g in range(d + 1):
        if D == 2:
            for k1 in range(g, -1, -1):
                out.append((k1, g - k1))
        else:
            for k1 in range(g, -1, -1):
                for k2 in range(g - k1, -1, -1):
                    out.append((k1, k2, g - k1 - k2))
    return out


# --------------------------------------------------------------------------
# univariate Legendre polynomials (floating point evaluation)


def legendre(k, x):
    """l_k(x) by Bonnet's recurrence; x array."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if k == 0:
        return p0
    p1 = x.copy()
    for j in range(1, k):
        p0, p1 = p1, ((2 * j + 1) * x * p1 - j * p0) / (j + 1)
    return p1


def legendre_deriv(k, x):
    """l_k'(x) from l_{k}' = sum over j = k-1, k-3, ... of (2j+1) l_j(x)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for j in range(k - 1, -1, -2):
        out = out + (2 * j + 1) * legendre(j, x)
    return out


def legendre_mass(D, d):
    """Diagonal mass M_l = prod_i 2/(2 k_i + 1)."""
    return np.array([np.prod([2.0 / (2 * k + 1) for k in e]) for e in mode_exponents(D, d)])


def legendre_values(D, d, xi):
    """Table V[p, l] = P_l(xi_p), xi[P, D]."""
    ex = mode_exponents(D, d)
    V = np.empty((xi.shape[0], len(ex)))
    for l, e in enumerate(ex):
        v = np.ones(xi.shape[0])
        for a in range(D):
            v = v * legendre(e[a], xi[:, a])
        V[:, l] = v
    return V


def legendre_grads(D, d, xi):
    """Table G[a, p, l] = dP_l/dxi_a (xi_p)."""
    ex = mode_exponents(D, d)
    G = np.empty((D, xi.shape[0], len(ex)))
    for a in range(D):
        for l, e in enumerate(ex):
            v = np.ones(xi.shape[0])
            for b in range(D):
                v = v * (legendre_deriv(e[b], xi[:, b]) if b == a else legendre(e[b], xi[:, b]))
            G[a, :, l] = v
    return G


# --------------------------------------------------------------------------
# exact polynomial algebra for the LDF generator.  A polynomial is a dict
# {exponent tuple (length 3): Fraction}.


def _padd(p, q, s=Fraction(1)):
    r = dict(p)
    for e, c in q.items():
        r[e] = r.get(e, Fraction(0)) + s * c
        if r[e] == 0:
            del r[e]
    return r


def _pscale(p, s):
    if s == 0:
        return {}
    return {e: c * s for e, c in p.items()}


def _pmul(p, q):
    r = {}
    for e1, c1 in p.items():
        for e2, c2 in q.items():
            e = tuple(a + b for a, b in zip(e1, e2))
            r[e] = r.get(e, Fraction(0)) + c1 * c2
    return {e: c for e, c in r.items() if c != 0}


def _pderiv(p, a):
    r = {}
    for e, c in p.items():
        if e[a] > 0:
            e2 = list(e)
            e2[a] -= 1
            r[tuple(e2)] = r.get(tuple(e2), Fraction(0)) + c * e[a]
    return {e: c for e, c in r.items() if c != 0}


def _pdegree(p):
    return max((sum(e) for e in p), default=-1)


@lru_cache(maxsize=None)
def _legendre_coeffs(k):
    """Exact monomial coefficients of l_k (list, index = power)."""
    if k == 0:
        return (Fraction(1),)
    p0, p1 = [Fraction(1)], [Fraction(0), Fraction(1)]
    for j in range(1, k):
        nxt = [Fraction(0)] * (j + 2)
        for i, c in enumerate(p1):
            nxt[i + 1] += Fraction(2 * j + 1, j + 1) * c
        for i, c in enumerate(p0):
            nxt[i] -= Fraction(j, j + 1) * c
        p0, p1 = p1, nxt
    return tuple(p1)


def _legendre_product_poly(e):
    """Exact P_e(xi) as a polynomial dict over 3 variables."""
    p = {(0, 0, 0): Fraction(1)}
    for a, k in enumerate(e):
        fac = {}
        for i, c in enumerate(_legendre_coeffs(k)):
            if c != 0:
                ex = [0, 0, 0]
                ex[a] = i
                fac[tuple(ex)] = c
        p = _pmul(p, fac)
    return p


def _int_monomial(e, D):
    """Exact integral of xi^e over [-1,1]^D."""
    r = Fraction(1)
    for a in range(D):
        k = e[a]
        if k % 2:
            return Fraction(0)
        r *= Fraction(2, k + 1)
    return r


def _vinner(V, W, D):
    """<V, W> = int_{[-1,1]^D} sum_c V_c W_c (App. A)."""
    s = Fraction(0)
    for c in range(len(V)):
        for e1, c1 in V[c].items():
            for e2, c2 in W[c].items():
                s += c1 * c2 * _int_monomial(tuple(a + b for a, b in zip(e1, e2)), D)
    return s


def _curl(V):
    """curl of a 3-vector of polynomials."""
    return [
        _padd(_pderiv(V[2], 1), _pderiv(V[1], 2), Fraction(-1)),
        _padd(_pderiv(V[0], 2), _pderiv(V[2], 0), Fraction(-1)),
        _padd(_pderiv(V[1], 0), _pderiv(V[0], 1), Fraction(-1)),
    ]


@lru_cache(maxsize=None)
def ldf_basis_exact(D, d, pool="legendre"):
    """Exact LDF basis: tuple of N_div vectors, each a tuple of D polynomial dicts
    (variables xi1..xi3, xi3 absent in 2-D).  App. A generation procedure."""
    if pool == "legendre":
        Qs = [_legendre_product_poly(tuple(e) + (0,) * (3 - D)) for e in mode_exponents(D, d + 1)]
    elif pool == "monomial":
        Qs = [{tuple(e) + (0,) * (3 - D): Fraction(1)} for e in mode_exponents(D, d + 1)]
    else:
        raise ValueError(pool)
    cands = []
    if D == 3:
        for comp in range(3):
            for Q in Qs:
                V = [{}, {}, {}]
                V[comp] = Q
                cands.append(_curl(V))
    else:
        for Q in Qs:
            c = _curl([{}, {}, Q])
            cands.append([c[0], c[1]])
    cands = [c for c in cands if any(len(p) for p in c)]
    cands.sort(key=lambda c: max(_pdegree(p) for p in c))  # stable
    basis, norms = [], []
    target = n_div(D, d)
    for c in cands:
        r = [dict(p) for p in c]
        for b, nb in zip(basis, norms):
            proj = _vinner(c, b, D) / nb
            if proj != 0:
                r = [_padd(rp, bp, -proj) for rp, bp in zip(r, b)]
        if any(len(p) for p in r):
            nr = _vinner(r, r, D)
            basis.append(r)
            norms.append(nr)
            if len(basis) == target:
                break
    if len(basis) != target:
        raise RuntimeError("LDF generator did not reach N_div")
    return tuple(tuple(v) for v in basis), tuple(norms)


def _peval(p, xi):
    out = np.zeros(xi.shape[0])
    for e, c in p.items():
        term = np.full(xi.shape[0], float(c))
        for a in range(xi.shape[1]):
            if e[a]:
                term = term * xi[:, a] ** e[a]
        out += term
    return out


def ldf_mass(D, d):
    basis, norms = ldf_basis_exact(D, d)
    return np.array([float(n) for n in norms])


def ldf_values(D, d, xi):
    """Table Phi[c, p, l] = component c of LDF function l at xi_p."""
    basis, _ = ldf_basis_exact(D, d)
    out = np.empty((D, xi.shape[0], len(basis)))
    for l, V in enumerate(basis):
        for c in range(D):
            out[c, :, l] = _peval(V[c], xi)
    return out


def ldf_grads(D, d, xi):
    """Table dPhi[a, c, p, l] = d Phi_{l,c} / d xi_a at xi_p."""
    basis, _ = ldf_basis_exact(D, d)
    out = np.empty((D, D, xi.shape[0], len(basis)))
    for l, V in enumerate(basis):
        for c in range(D):
            for a in range(D):
                out[a, c, :, l] = _peval(_pderiv(V[c], a), xi)
    return out


def ldf_degrees(D, d):
    basis, _ = ldf_basis_exact(D, d)
    return [max(_pdegree(p) for p in V) for V in basis]


def ldf_divergence_exact(V):
    """Exact divergence polynomial of an LDF vector (for the zero-divergence pin)."""
    r = {}
    for a, p in enumerate(V):
        r = _padd(r, _pderiv(p, a))
    return r


def ldf_project_exact(D, d, U):
    """Exact projections int U . Phi_l for a vector polynomial U (tuple of D dicts)."""
    basis, _ = ldf_basis_exact(D, d)
    return [_vinner(list(U), list(V), D) for V in basis]
