"""Pins of the oracle's Powell scheme (no GPU): the face term of
Sec. 4.1.3 (eq. powell-src-face with q-dagger = q(<u>_K), eq. powellq-average,
B^n_F of eq. bxface-average-alfven) and the time-step cap of Sec. 4.1.4
(eq. powell_dt with |div B|_K from the face-jump part of eq. divb-cell).

* brute force: the whole right-hand side on 2^3 / 3^3 periodic grids written
  cell by cell and face by face with outward normals, the LDF functions
  evaluated straight from their exact rational polynomials, cell averages by
  quadrature, and a normal-field jump of O(0.1) at every face;
* an integral identity: on a periodic grid the face fluxes cancel in the
  totals, so the total rate of change of momentum and energy is the Powell
  term alone, -sum_K q(<u>_K) * (face integral of B^n_F - B^n_K), which a
  state with rho and B constant per cell gives in closed form;
* the cap: for the same kind of state with a small eta, the step is
  eta E / (|div B|_K |v.B|) of the limiting cell, worked out face by face.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import basis as Bm
from oracle import dg
from oracle import physics as ph
from oracle.quadrature import tensor_rule

G = 5.0 / 3.0
LEG = np.polynomial.legendre


# ---------------------------------------------------------------- helpers


def _poly_eval(p, pts):
    """Value of an exact polynomial {exponents: Fraction} at pts [P, 3]."""
    out = np.zeros(pts.shape[0])
    for e, c in p.items():
        out += float(c) * pts[:, 0] ** e[0] * pts[:, 1] ** e[1] * pts[:, 2] ** e[2]
    return out


def _poly_deriv_eval(p, a, pts):
    out = np.zeros(pts.shape[0])
    for e, c in p.items():
        if e[a] == 0:
            continue
        ee = list(e)
        k = ee[a]
        ee[a] -= 1
        out += float(c) * k * pts[:, 0] ** ee[0] * pts[:, 1] ** ee[1] * pts[:, 2] ** ee[2]
    return out


class _Brute:
    """Direct evaluation of the Powell/LDF scheme's polynomials (3-D)."""

    def __init__(self, d):
        self.d = d
        self.ex = Bm.mode_exponents(3, d)
        self.nm = len(self.ex)
        self.ldf, _ = Bm.ldf_basis_exact(3, d)
        self.nd = len(self.ldf)
        self.xg, self.wg = LEG.leggauss(d + 1)
        g = np.meshgrid(self.xg, self.xg, self.xg, indexing="ij")
        self.vpts = np.stack([x.ravel() for x in g], 1)
        self.vw = np.prod(np.meshgrid(self.wg, self.wg, self.wg, indexing="ij"), axis=0).ravel()
        t = np.meshgrid(self.xg, self.xg, indexing="ij")
        self.tpts = np.stack([x.ravel() for x in t], 1)
        self.tw = np.prod(np.meshgrid(self.wg, self.wg, indexing="ij"), axis=0).ravel()
        # masses by quadrature exact for the squared polynomials
        xh, wh = LEG.leggauss(d + 3)
        gh = np.meshgrid(xh, xh, xh, indexing="ij")
        ph_ = np.stack([x.ravel() for x in gh], 1)
        wh3 = np.prod(np.meshgrid(wh, wh, wh, indexing="ij"), axis=0).ravel()
        self.mleg = np.array([np.sum(wh3 * self.leg(l, ph_) ** 2) for l in range(self.nm)])
        self.mldf = np.array([np.sum(wh3 * sum(_poly_eval(V[c], ph_) ** 2 for c in range(3))) for V in self.ldf])

    def leg(self, l, pts):
        c = np.zeros((self.d + 1,) * 3)
        c[self.ex[l]] = 1.0
        return LEG.legval3d(pts[:, 0], pts[:, 1], pts[:, 2], c)

    def dleg(self, l, a, pts):
        c = np.zeros((self.d + 1,) * 3)
        c[self.ex[l]] = 1.0
        if self.ex[l][a] == 0:
            return np.zeros(pts.shape[0])
        return LEG.legval3d(pts[:, 0], pts[:, 1], pts[:, 2], LEG.legder(c, axis=a))

    def state(self, wc, pts):
        """Conserved 8-component state of one cell's weights wc at pts."""
        U = np.zeros((8, pts.shape[0]))
        for v in range(5):
            for l in range(self.nm):
                U[v] += wc[v * self.nm + l] * self.leg(l, pts)
        o = 5 * self.nm
        for l, V in enumerate(self.ldf):
            for c in range(3):
                U[ph.B1 + c] += wc[o + l] * _poly_eval(V[c], pts)
        return U

    def test_products(self, vals, pts, weights):
        """sum_r weights_r vals[:, r] . phi_m(r) for every mode m (8-comp vals)."""
        out = np.zeros(5 * self.nm + self.nd)
        for v in range(5):
            for l in range(self.nm):
                out[v * self.nm + l] = np.sum(weights * vals[v] * self.leg(l, pts))
        o = 5 * self.nm
        for l, V in enumerate(self.ldf):
            out[o + l] = sum(np.sum(weights * vals[ph.B1 + c] * _poly_eval(V[c], pts)) for c in range(3))
        return out


def _brute_rhs_powell(d, n, w, interp=False):
    """R/M of eq. wdot with the Powell face term on an n^3 periodic grid of
    the unit box, written cell by cell: volume integral with the analytic
    flux, face fluxes of both faces of every axis with the outward normal,
    and -(2/h) sum_faces sum_r w_r (q(<u>_K) . phi_l)(B^n_F - B^n_K) with the
    outward normal field component.  Shares only the pointwise physics."""
    br = _Brute(d)
    h = 1.0 / n
    C = n ** 3
    R = np.zeros((C, 5 * br.nm + br.nd))

    def idx(ijk):
        return sum((ijk[a] % n) * n ** a for a in range(3))

    for cell in range(C):
        ijk = [(cell // n ** a) % n for a in range(3)]
        U = br.state(w[cell], br.vpts)
        ubar = (U * br.vw).sum(axis=1) / 8.0          # cell average by quadrature
        q = ph.powell_q(ubar[:, None])[:, 0]           # (0, B, v.B, v)
        # volume: sum_q w_q sum_a f_a(u_q) . d_a phi_l
        for a in range(3):
            F = ph.flux(U, a, G)
            for v in range(5):
                for l in range(br.nm):
                    R[cell, v * br.nm + l] += (2 / h) * np.sum(br.vw * F[v] * br.dleg(l, a, br.vpts))
            o = 5 * br.nm
            for l, V in enumerate(br.ldf):
                R[cell, o + l] += (2 / h) * sum(np.sum(br.vw * F[ph.B1 + c] * _poly_deriv_eval(V[c], a, br.vpts))
                                                for c in range(3))
        # faces with outward normal side * e_a
        for a in range(3):
            for side in (+1, -1):
                nb = list(ijk)
                nb[a] += side
                pin = np.insert(br.tpts, a, side, axis=1)
                pout = np.insert(br.tpts, a, -side, axis=1)
                Ui, Uo = br.state(w[cell], pin), br.state(w[idx(nb)], pout)
                if side > 0:
                    F, bnF, vF, BF = ph.numerical_flux(Ui, Uo, a, G, state=True)
                else:
                    F, bnF, vF, BF = ph.numerical_flux(Uo, Ui, a, G, state=True)
                R[cell] -= side * (2 / h) * br.test_products(F, pin, br.tw)
                jump = side * (bnF - Ui[ph.B1 + a])     # (B_F - B_K) . n
                qd = ph.powell_q_interp(Ui, vF, BF) if interp else q[:, None]
                R[cell] -= (2 / h) * br.test_products(qd * jump[None, :], pin, br.tw)
    M = np.concatenate([np.tile(br.mleg, 5), br.mldf])
    return R / M[None, :]


def _perturbed_powell_state(s, seed):
    rng = np.random.default_rng(seed)
    w = s.project(dg.conserved_field(wl.Smooth(31, 3), G, 8))
    nl = 5 * s.n
    w[:, :nl] += 0.02 * rng.normal(size=(s.mesh.ncells, nl)) * (np.arange(nl) % s.n != 0)
    # normal-field jumps of O(0.1) at every face
    w[:, nl:] += 0.05 * rng.normal(size=(s.mesh.ncells, s.nldf))
    return w


@pytest.mark.parametrize("d,n,qmode", [(1, 3, "mean"), (2, 2, "mean"), (1, 3, "interp"), (2, 2, "interp")])
def test_powell_rhs_matches_brute_force(d, n, qmode):
    s = dg.DG(dg.Mesh.uniform(3, n), d, divb=dg.POWELL, powell_q=qmode)
    w = _perturbed_powell_state(s, 40 + d)
    r = s.rhs(w)
    rb = _brute_rhs_powell(d, n, w, interp=qmode == "interp")
    # the jumps are really there: the Powell part is a sizable share of R
    assert np.abs(rb).max() > 0.1
    assert np.allclose(r, rb, rtol=1e-12, atol=1e-12 * np.abs(rb).max())


# ---------------------------------------------------------------- piecewise-constant states


def _blocky(n, seed):
    """rho and B constant per cell (random), v and p uniform."""
    rng = np.random.default_rng(seed)
    C = n ** 3
    rho = rng.uniform(0.6, 1.6, C)
    B = rng.normal(0.0, 0.6, (3, C))
    v = np.array([0.3, -0.2, 0.15])
    p = 1.1

    def cell_of(x):
        ijk = np.floor(x * n).astype(np.int64) % n
        return ijk[:, 0] + n * (ijk[:, 1] + n * ijk[:, 2])

    def field(x):
        c = cell_of(x)
        P = x.shape[0]
        return {"rho": rho[c], "v": [np.full(P, v[0]), np.full(P, v[1]), np.full(P, v[2])],
                "p": np.full(P, p), "B": [B[0][c], B[1][c], B[2][c]]}
    return field, rho, B, v, p


def _face_jumps(n, rho, B):
    """For every cell and face (axis a, side s): the outward jump
    (B_F - B_K) . n with B^n_F weighted by 1/sqrt(rho) (eq.
    bxface-average-alfven), computed face by face."""
    C = n ** 3
    J = np.zeros((C, 3, 2))
    for c in range(C):
        ijk = [(c // n ** a) % n for a in range(3)]
        for a in range(3):
            for k, side in enumerate((-1, +1)):
                nb = list(ijk)
                nb[a] = (nb[a] + side) % n
                o = nb[0] + n * (nb[1] + n * nb[2])
                lo, hi = (o, c) if side < 0 else (c, o)     # lower and upper cell of the face
                wl_, wh_ = 1 / math.sqrt(rho[lo]), 1 / math.sqrt(rho[hi])
                bF = (B[a][lo] * wl_ + B[a][hi] * wh_) / (wl_ + wh_)
                J[c, a, k] = side * (bF - B[a][c])
    return J


@pytest.mark.parametrize("d", [1, 2])
def test_powell_total_source_identity(d):
    n = 3
    h = 1.0 / n
    field, rho, B, v, p = _blocky(n, 7 + d)
    s = dg.DG(dg.Mesh.uniform(3, n), d, divb=dg.POWELL)
    w = s.project(dg.conserved_field(field, G, 8))
    r = s.rhs(w)
    J = _face_jumps(n, rho, B)
    area = h * h
    jsum = J.sum(axis=(1, 2)) * area                   # face integral of (B_F - B_K).n per cell
    vol = h ** 3
    # totals of the Legendre blocks (mode 0 is the cell mean)
    tot = np.array([(r[:, k * s.n] * vol).sum() for k in range(5)])
    exp_m = -np.array([(B[c] * jsum).sum() for c in range(3)])
    exp_E = -((v[0] * B[0] + v[1] * B[1] + v[2] * B[2]) * jsum).sum()
    scale = np.abs(B).max() * np.abs(jsum).max() * n ** 3
    assert abs(tot[0]) < 1e-13 * scale
    assert np.allclose(tot[1:4], exp_m, rtol=1e-12, atol=1e-13 * scale)
    assert math.isclose(tot[4], exp_E, rel_tol=1e-12, abs_tol=1e-13 * scale)
    assert np.abs(exp_m).max() > 0.1                   # the identity is not trivially 0 = 0
    # magnetic field: q_B = v is uniform, so the jumps of each face cancel in the total
    xq, wq = tensor_rule(d + 2, 3)
    Phi = Bm.ldf_values(3, d, xq)
    mean = np.einsum("q,cql->cl", wq, Phi) / 8.0
    totB = (r[:, 5 * s.n:] @ mean.T).sum(axis=0) * vol
    assert np.abs(totB).max() < 1e-13 * scale


def test_powell_dt_cap_binds_and_matches_hand_value():
    n, d = 3, 2
    h = 1.0 / n
    field, rho, B, v, p = _blocky(n, 21)
    eta = 1e-4
    s = dg.DG(dg.Mesh.uniform(3, n), d, divb=dg.POWELL, powell_eta=eta)
    w = s.project(dg.conserved_field(field, G, 8))
    dt, ch, kappa = s.timestep(w)
    # eq. cfl by hand: the state is constant inside each cell
    c = np.sqrt((G * p + (B ** 2).sum(axis=0)) / rho)
    dt_cfl = 0.3 / (2 * d + 1) * np.min(h / (np.abs(v).sum() + 3 * c))
    # eq. powell_dt with |div B|_K = (1/V_K) int |B_F - B_K| dS
    J = _face_jumps(n, rho, B)
    divb = np.abs(J).sum(axis=(1, 2)) * h * h / h ** 3
    E = p / (G - 1) + 0.5 * rho * (v ** 2).sum() + 0.5 * (B ** 2).sum(axis=0)
    vB = np.abs(v[0] * B[0] + v[1] * B[1] + v[2] * B[2])
    cap = np.min(eta * E / (divb * vB))
    assert cap < 0.5 * dt_cfl                          # the cap binds
    assert math.isclose(dt, cap, rel_tol=1e-12)
    # with the paper's eta = 0.2 the same state is CFL-limited
    s2 = dg.DG(dg.Mesh.uniform(3, n), d, divb=dg.POWELL)
    assert math.isclose(s2.timestep(w)[0], min(dt_cfl, cap * 0.2 / eta), rel_tol=1e-12)


def test_interpolated_q_differs_from_the_mean_and_conserves_mass():
    s = dg.DG(dg.Mesh.uniform(3, 3), 1, divb=dg.POWELL)
    si = dg.DG(dg.Mesh.uniform(3, 3), 1, divb=dg.POWELL, powell_q="interp")
    w = _perturbed_powell_state(s, 5)
    r, ri = s.rhs(w), si.rhs(w)
    vol = s.mesh.h ** 3
    assert abs((ri[:, 0] * vol).sum()) < 1e-13
    # the two q-daggers give different Powell terms in momentum and energy
    assert np.abs(ri[:, s.n:5 * s.n] - r[:, s.n:5 * s.n]).max() > 1e-3 * np.abs(r).max()
    # and the same fluxes: the mass equation is untouched
    assert np.allclose(ri[:, :s.n], r[:, :s.n], rtol=0, atol=1e-13 * np.abs(r[:, :s.n]).max())
