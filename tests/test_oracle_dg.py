"""Pins of the oracle's DG operator, time step and SSP-RK3 (no GPU):
free-stream preservation, conservation, closed-form GLM damping, brute-force
quadrature on tiny grids, and d+1 convergence on the travelling Alfven wave."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dg
from oracle import physics as ph
from oracle.quadrature import tensor_rule

G = 5.0 / 3.0


def uniform_state(nvar):
    u = np.array([1.3, 0.2, -0.1, 0.3, 4.0, 0.7, -0.4, 0.5, 0.25])[:nvar]
    return lambda x: np.tile(u[:, None], (1, x.shape[0]))


@pytest.mark.parametrize("D,d,divb", [(2, 1, dg.GLM), (2, 3, dg.GLM), (3, 2, dg.GLM), (3, 1, dg.POWELL),
                                      (3, 2, dg.POWELL)])
def test_free_stream_preserved(D, d, divb):
    m = dg.Mesh.uniform(D, 3)
    s = dg.DG(m, d, divb=divb)
    w = s.project(uniform_state(s.nvar))
    r = s.rhs(w, ch=1.5, kappa=0.0)
    scale = (2.0 / m.h[0]) * 10.0
    assert np.abs(r).max() < 1e-14 * scale * 10


@pytest.mark.parametrize("D,d", [(2, 1), (3, 1)])
def test_glm_conservation_over_steps(D, d):
    m = dg.Mesh.uniform(D, 8 if D == 2 else 4)
    s = dg.DG(m, d)
    w = s.project(dg.conserved_field(wl.Smooth(11, D), G, 9))
    vol = m.h ** D
    tot0 = (w[:, ::s.n] * vol[:, None]).sum(0)
    for _ in range(3):
        w, dt, ch, k = s.step(w)
    tot1 = (w[:, ::s.n] * vol[:, None]).sum(0)
    scale = np.abs(w[:, ::s.n]).max(0)
    # rho, m, E, B conserved to rounding; psi decays
    assert np.all(np.abs(tot1 - tot0)[:8] < 1e-14 * np.maximum(scale[:8], 1.0))


def test_powell_conserves_mass_only():
    m = dg.Mesh.uniform(3, 4)
    s = dg.DG(m, 1, divb=dg.POWELL)
    w = s.project(dg.conserved_field(wl.Smooth(12, 3), G, 8))
    # add a jump in the normal field by perturbing the LDF weights cell by cell
    rng = np.random.default_rng(0)
    w[:, 5 * s.n:] += 0.05 * rng.normal(size=(m.ncells, s.nldf))
    r = s.rhs(w)
    vol = m.h ** 3
    assert abs((r[:, 0] * vol).sum()) < 1e-14
    # the Powell terms inject momentum/energy when div B != 0 at faces
    assert abs((r[:, s.n] * vol).sum()) > 1e-8 or abs((r[:, 4 * s.n] * vol).sum()) > 1e-8


def test_glm_damping_closed_form():
    # uniform B and psi: d psi/dt = -kappa psi exactly; one SSP-RK3 step gives
    # psi0 (1 - z + z^2/2 - z^3/6), z = kappa dt
    m = dg.Mesh.uniform(2, 4)
    s = dg.DG(m, 2)
    psi0 = 0.37
    u = np.array([1.0, 0.1, 0.2, 0.0, 2.0, 0.3, 0.4, 0.1, psi0])
    w = s.project(lambda x: np.tile(u[:, None], (1, x.shape[0])))
    w1, dt, ch, kappa = s.step(w)
    z = kappa * dt
    assert z > 0.01
    assert np.allclose(w1[:, 8 * s.n], psi0 * (1 - z + z * z / 2 - z ** 3 / 6), rtol=1e-13)
    assert np.abs(w1[:, 8 * s.n + 1:]).max() < 1e-14


def test_timestep_formula_uniform_state():
    # eq. cfl with c = sqrt(c_s^2 + c_A^2) on a uniform state, and c_h, kappa readings
    m = dg.Mesh.uniform(3, 4)
    s = dg.DG(m, 2, cfl=0.3)
    u = np.array([1.3, 0.2, -0.1, 0.3, 4.0, 0.7, -0.4, 0.5, 0.0])
    w = s.project(lambda x: np.tile(u[:, None], (1, x.shape[0])))
    dt, ch, kappa = s.timestep(w)
    rho, v = u[0], u[1:4] / u[0]
    Bv = u[5:8]
    p = (G - 1) * (u[4] - 0.5 * rho * v @ v - 0.5 * Bv @ Bv)
    c = math.sqrt(G * p / rho + Bv @ Bv / rho)
    ssum = np.abs(v).sum() + 3 * c
    assert np.isclose(dt, 0.3 / 5 * m.h[0] / ssum, rtol=1e-13)
    assert np.isclose(ch, (0.6 / 0.3) * ssum / 3, rtol=1e-13)
    assert np.isclose(kappa, min(ch / 0.18, 1 / (3 * dt)), rtol=1e-13)


# ---------------------------------------------------------------- brute force


def _brute_rhs(D, d, n, w, ch, kappa):
    """R of eq. wdot on an n^D periodic grid, written with numpy's own Legendre
    series evaluation (legval2d/3d, legder) and numpy's Gauss-Legendre rule,
    cell by cell and face by face in plain loops.  Shares the pointwise physics
    only."""
    from oracle import basis as Bm
    L = np.polynomial.legendre
    h = 1.0 / n
    ex = Bm.mode_exponents(D, d)
    nm = len(ex)
    xg, wg = L.leggauss(d + 1)

    def coeff(cell, v):
        c = np.zeros((d + 1,) * D)
        for l, e in enumerate(ex):
            c[e] = w[cell, v * nm + l]
        return c

    def ev(c, pts):
        return (L.legval2d(pts[:, 0], pts[:, 1], c) if D == 2 else
                L.legval3d(pts[:, 0], pts[:, 1], pts[:, 2], c))

    def state(cell, pts):
        return np.stack([ev(coeff(cell, v), pts) for v in range(9)])

    grids = np.meshgrid(*([xg] * D), indexing="ij")
    vpts = np.stack([g.ravel() for g in grids], 1)
    vw = np.prod(np.meshgrid(*([wg] * D), indexing="ij"), axis=0).ravel()
    C = n ** D
    R = np.zeros((C, 9 * nm))
    def idx(ijk):
        return sum((ijk[a] % n) * n ** a for a in range(D))
    for cell in range(C):
        ijk = [(cell // n ** a) % n for a in range(D)]
        U = state(cell, vpts)
        for a in range(D):
            F = ph.flux(U, a, G, True, ch)
            for l, e in enumerate(ex):
                c = np.zeros((d + 1,) * D)
                c[e] = 1.0
                dphi = ev(L.legder(c, axis=a) if c.shape[a] > 1 else np.zeros_like(c), vpts)
                for v in range(9):
                    R[cell, v * nm + l] += (2 / h) * np.sum(vw * F[v] * dphi)
        # faces with outward normal +e_a and -e_a
        for a in range(D):
            tg = np.meshgrid(*([xg] * (D - 1)), indexing="ij")
            tp = np.stack([g.ravel() for g in tg], 1) if D > 1 else np.zeros((1, 0))
            tw = np.prod(np.meshgrid(*([wg] * (D - 1)), indexing="ij"), axis=0).ravel()
            for side in (+1, -1):
                nb = list(ijk)
                nb[a] += side
                pin = np.insert(tp, a, side, axis=1)
                pout = np.insert(tp, a, -side, axis=1)
                Ui, Uo = state(cell, pin), state(idx(nb), pout)
                if side > 0:
                    F, _ = ph.numerical_flux(Ui, Uo, a, G, True, ch)
                else:
                    F, _ = ph.numerical_flux(Uo, Ui, a, G, True, ch)
                for l, e in enumerate(ex):
                    c = np.zeros((d + 1,) * D)
                    c[e] = 1.0
                    phi = ev(c, pin)
                    for v in range(9):
                        R[cell, v * nm + l] -= side * (2 / h) * np.sum(tw * F[v] * phi)
        for l, e in enumerate(ex):
            M = np.prod([2.0 / (2 * k + 1) for k in e])
            R[cell, 8 * nm + l] -= kappa * M * w[cell, 8 * nm + l]
    Mv = np.array([np.prod([2.0 / (2 * k + 1) for k in e]) for e in ex])
    return R / np.tile(Mv, 9)[None, :]


@pytest.mark.parametrize("D,d,n", [(2, 1, 3), (2, 2, 2), (2, 3, 3), (3, 1, 2), (3, 2, 2)])
def test_rhs_matches_brute_force(D, d, n):
    m = dg.Mesh.uniform(D, n)
    s = dg.DG(m, d)
    rng = np.random.default_rng(100 + 10 * D + d)
    w = s.project(dg.conserved_field(wl.Smooth(21, D), G, 9))
    w = w + 0.02 * rng.normal(size=w.shape) * (np.arange(w.shape[1]) % s.n != 0)
    w[:, 8 * s.n:] = 0.05 * rng.normal(size=(m.ncells, s.n))
    ch, kappa = 2.3, 4.1
    r = s.rhs(w, ch, kappa)
    rb = _brute_rhs(D, d, n, w, ch, kappa)
    assert np.allclose(r, rb, rtol=1e-12, atol=1e-12 * np.abs(rb).max())


# ---------------------------------------------------------------- convergence


def _alfven_l1_error(n, d, tend=0.2):
    A = wl.Alfven2D()
    m = dg.Mesh.uniform(2, n, box=A.L)
    s = dg.DG(m, d, cfl=0.3)
    w = s.project(dg.conserved_field(A, G, 9))
    t = 0.0
    while t < tend - 1e-14:
        dt, ch, k = s.timestep(w)
        dt = min(dt, tend - t)
        if d == 3:  # keep the RK3 time error below the spatial error: dt ~ h^(4/3)
            dt = min(dt, 0.05 * (m.h[0] / A.L) ** (4 / 3))
        u1 = w + dt * s.rhs(w, ch, k)
        u2 = 0.75 * w + 0.25 * (u1 + dt * s.rhs(u1, ch, k))
        w = w / 3 + 2 / 3 * (u2 + dt * s.rhs(u2, ch, k))
        t += dt
    xq, wq = tensor_rule(d + 3, 2)
    U = s.nodal(w, xi=xq)
    x = m.centers[:, None, :] + 0.5 * m.h[:, None, None] * xq[None]
    exact = A(x.reshape(-1, 2), t=tend)["B"][0].reshape(U.shape[1], -1)
    return (np.abs(U[ph.B1] - exact) * wq).sum() / (4 * m.ncells)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_alfven_wave_convergence_order(d):
    # Sec. 5.2.3: travelling circularly polarised Alfven wave, order d+1
    e = [_alfven_l1_error(n, d) for n in (8, 16, 32)]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert orders[-1] >= d + 1 - 0.3, (e, orders)


def _alfven3d_l1_error(n, d, divb, tend=0.01):
    A = wl.Alfven3D()
    m = dg.Mesh.uniform(3, n)
    s = dg.DG(m, d, divb=divb)
    w = s.project(dg.conserved_field(A, G, s.nvar))
    t = 0.0
    while t < tend - 1e-14:
        dt, ch, k = s.timestep(w)
        dt = min(dt, tend - t)
        u1 = w + dt * s.rhs(w, ch, k)
        u2 = 0.75 * w + 0.25 * (u1 + dt * s.rhs(u1, ch, k))
        w = w / 3 + 2 / 3 * (u2 + dt * s.rhs(u2, ch, k))
        t += dt
    xq, wq = tensor_rule(d + 3, 3)
    U = s.nodal(w, xi=xq)
    x = m.centers[:, None, :] + 0.5 * m.h[:, None, None] * xq[None]
    exact = A(x.reshape(-1, 3), t=tend)["B"][0].reshape(U.shape[1], -1)
    return (np.abs(U[ph.B1] - exact) * wq).sum() / (8 * m.ncells)


def test_alfven3d_powell_ldf_convergence():
    # Sec. 5.2.4: 3-D circularly polarised Alfven wave, Powell scheme on the LDF basis
    e = [_alfven3d_l1_error(n, 1, dg.POWELL) for n in (4, 8, 16)]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert orders[-1] >= 1.7, (e, orders)
