"""Pins of the oracle's SSP Runge-Kutta schemes of order 1-4 (Sec. 3.6):

* the Shu-Osher coefficients, turned into a Butcher tableau, satisfy the
  classical order conditions of each scheme's order (1, 2, 3, and all eight
  conditions of order 4 for the five-stage scheme) and not those of the
  next order;
* they are SSP: every coefficient is non-negative and each stage is a convex
  combination (alpha rows sum to 1);
* the linear GLM damping dpsi/dt = -kappa psi is advanced by the truncated
  exponential of each order (orders 1-3: the scheme's stability polynomial
  is the Taylor polynomial);
* on a fixed DG operator (smooth 2-D state, fixed c_h and kappa) the error
  against a fine-step reference falls with the scheme's order in dt.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dg

G = 5.0 / 3.0


def butcher(stages):
    alpha, beta = dg.ssp_rk(stages)
    s = len(alpha)
    A = np.zeros((s + 1, s + 1))   # stage i = u^n + dt sum_k A[i, k] L(u_k)
    for i in range(1, s + 1):
        for j in range(i):
            A[i] += alpha[i - 1][j] * A[j]
            A[i, j] += beta[i - 1][j]
    return A[:s, :s], A[s, :s], A[:s].sum(axis=1)


def order_conditions(A, b, c):
    """Residuals of the order conditions of orders 1..4 (rooted trees)."""
    return {
        1: [b.sum() - 1],
        2: [b @ c - 1 / 2],
        3: [b @ c ** 2 - 1 / 3, b @ A @ c - 1 / 6],
        4: [b @ c ** 3 - 1 / 4, (b * c) @ A @ c - 1 / 8, b @ A @ c ** 2 - 1 / 12, b @ A @ A @ c - 1 / 24],
    }


@pytest.mark.parametrize("stages,order", [(1, 1), (2, 2), (3, 3), (5, 4)])
def test_ssp_rk_order_conditions(stages, order):
    A, b, c = butcher(stages)
    res = order_conditions(A, b, c)
    for p in range(1, order + 1):
        assert np.all(np.abs(res[p]) < 1e-14), (p, res[p])
    if order < 4:
        assert np.max(np.abs(res[order + 1])) > 1e-3   # not of higher order


@pytest.mark.parametrize("stages", [1, 2, 3, 5])
def test_ssp_rk_coefficients_are_convex(stages):
    alpha, beta = dg.ssp_rk(stages)
    for arow, brow in zip(alpha, beta):
        assert min(arow) >= 0.0 and min(brow) >= 0.0
        assert abs(sum(arow) - 1.0) < 2e-15
        # a stage uses dt L(u_j) only together with u_j (Shu-Osher form)
        for a, b_ in zip(arow, brow):
            assert b_ == 0.0 or a > 0.0 or (len(arow) == 1)


@pytest.mark.parametrize("stages", [1, 2, 3])
def test_glm_damping_follows_the_taylor_polynomial(stages):
    m = dg.Mesh.uniform(2, 4)
    s = dg.DG(m, 2)
    psi0 = 0.37
    u = np.array([1.0, 0.1, 0.2, 0.0, 2.0, 0.3, 0.4, 0.1, psi0])
    w = s.project(lambda x: np.tile(u[:, None], (1, x.shape[0])))
    w1, dt, ch, kappa = s.step(w, rk=stages)
    z = kappa * dt
    assert z > 0.01
    expect = sum((-z) ** k / math.factorial(k) for k in range(stages + 1))
    assert np.allclose(w1[:, 8 * s.n], psi0 * expect, rtol=1e-13)


def _integrate(s, w, T, nsteps, stages, ch, kappa):
    alpha, beta = dg.ssp_rk(stages)
    dt = T / nsteps
    for _ in range(nsteps):
        us, dls = [w], []
        for i in range(len(alpha)):
            dls.append(dt * s.rhs(us[-1], ch, kappa))
            us.append(sum(alpha[i][j] * us[j] + beta[i][j] * dls[j] for j in range(i + 1)))
        w = us[-1]
    return w


@pytest.mark.parametrize("stages,order", [(1, 1), (2, 2), (3, 3), (5, 4)])
def test_temporal_order_on_a_fixed_dg_operator(stages, order):
    s = dg.DG(dg.Mesh.uniform(2, 6), 1)
    w0 = s.project(dg.conserved_field(wl.Smooth(71, 2), G, 9))
    dt0, ch, kappa = s.timestep(w0)
    T = 8 * dt0
    ref = _integrate(s, w0, T, 128, 5, ch, kappa)
    errs = [np.abs(_integrate(s, w0, T, n, stages, ch, kappa) - ref).max() for n in (8, 16, 32)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > order - 0.25, (errs, rates)
    assert rates[-1] < order + 0.8
