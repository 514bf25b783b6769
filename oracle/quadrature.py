"""Gauss-Legendre quadrature (oracle; test infrastructure only).

Sec. 3.5 ("Semi-discrete DG scheme"): volume and face integrals use
Gauss-Legendre quadrature with d+1 nodes per dimension, exact for polynomials
of degree <= 2d+1.  Sec. 5.2.1 (L^p error norm, eq. lp_norm) uses d+3 nodes.

The nodes are the roots of the Legendre polynomial P_n, found by Newton's
method from the Chebyshev-like initial guess cos(pi (i + 3/4) / (n + 1/2));
the weights are 2 / ((1 - x^2) P_n'(x)^2) (textbook Gauss-Legendre).
"""
import math

import numpy as np


def _legendre_and_derivative(n, x):
    """P_n(x) and P_n'(x) by Bonnet's recurrence (k+1)P_{k+1} = (2k+1)xP_k - kP_{k-1}."""
    p0, p1 = 1.0, x
    if n == 0:
        return 1.0, 0.0
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    return p1, dp


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [-1, 1]; nodes ascending."""
    if n < 1:
        raise ValueError("n >= 1")
    nodes = np.empty(n)
    weights = np.empty(n)
    for i in range(n):
        x = math.cos(math.pi * (i + 0.75) / (n + 0.5))
        for _ in range(100):
            p, dp = _legendre_and_derivative(n, x)
            dx = p / dp
            x -= dx
            if abs(dx) < 1e-17:
                break
        p, dp = _legendre_and_derivative(n, x)
        nodes[i] = x
        weights[i] = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(nodes)
    nodes = nodes[order]
    weights = weights[order]
    # exact symmetry of the rule
    nodes = 0.5 * (nodes - nodes[::-1])
    weights = 0.5 * (weights + weights[::-1])
    if n % 2 == 1:
        nodes[n // 2] = 0.0
    return nodes, weights


def tensor_rule(n, D):
    """Tensor-product rule on [-1,1]^D.  Point index q = q0 + n*(q1 + n*q2),
    i.e. the first coordinate runs fastest.  Returns (xi[Q, D], w[Q])."""
    x, w = gauss_legendre(n)
    if D == 1:
        return x[:, None].copy(), w.copy()
    if D == 2:
        q1, q0 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        q0, q1 = q0.ravel(), q1.ravel()
        return np.stack([x[q0], x[q1]], axis=1), w[q0] * w[q1]
    if D == 3:
        q2, q1, q0 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        q0, q1, q2 = q0.ravel(), q1.ravel(), q2.ravel()
        return np.stack([x[q0], x[q1], x[q2]], axis=1), w[q0] * w[q1] * w[q2]
    raise ValueError("D in 1..3")
