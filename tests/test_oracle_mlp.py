"""Pins of the oracle's learned-indicator network (no GPU): analytic
gradients against central finite differences in FP64, GELU against its
closed form, bf16 rounding against exact ties, and feature construction."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dg, mlp


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0])
    r = mlp.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: round to even (1.0); 1 + 3*2^-8 -> 1 + 2^-6
    assert np.array_equal(r, [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0])


def test_gelu_closed_form():
    for x in (-3.0, -0.5, 0.0, 0.7, 2.0):
        Phi = 0.5 * (1 + math.erf(x / math.sqrt(2)))
        assert mlp.gelu(np.array([x]))[0] == pytest.approx(x * Phi, abs=1e-15)
        h = 1e-6
        fd = (mlp.gelu(np.array([x + h]))[0] - mlp.gelu(np.array([x - h]))[0]) / (2 * h)
        assert mlp.gelu_grad(np.array([x]))[0] == pytest.approx(fd, rel=1e-8, abs=1e-10)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = mlp.init_params(1)
    X = rng.normal(size=(12, 256))
    y = (rng.uniform(size=12) > 0.5).astype(float)
    loss, G = mlp.backward(P, X, y)
    for i, idx in [(0, (3, 5)), (0, (255, 63)), (1, (7,)), (2, (10, 20)), (4, (0, 1)), (6, (5, 0)), (7, (0,))]:
        Pp = [p.copy() for p in P]
        Pm = [p.copy() for p in P]
        h = 1e-6
        Pp[i][idx] += h
        Pm[i][idx] -= h
        fd = (mlp.bce(mlp.forward(Pp, X)[0], y) - mlp.bce(mlp.forward(Pm, X)[0], y)) / (2 * h)
        assert G[i][idx] == pytest.approx(fd, rel=1e-6, abs=1e-10), (i, idx)


def test_bf16_mode_is_close_to_fp64():
    rng = np.random.default_rng(2)
    P = mlp.init_params(3)
    X = rng.normal(size=(64, 256))
    y = (rng.uniform(size=64) > 0.7).astype(float)
    l64, G64 = mlp.backward(P, X, y)
    l16, G16 = mlp.backward(P, X, y, bf16=True)
    assert abs(l64 - l16) < 1e-2 * l64
    for a, b in zip(G64, G16):
        assert np.abs(a - b).max() <= 3e-2 * np.abs(a).max() + 1e-8


def test_features_layout():
    s = dg.DG(dg.Mesh.uniform(3, 4), 3)
    w = s.project(dg.conserved_field(wl.Blast(2000), 5 / 3, 9))
    sig = mlp.feature_scale(s, w)
    F = mlp.features(s, w, sig)
    assert F.shape == (64, 256)
    assert np.all(F[:, 234:] == 0.0)
    means = s.cell_means(w)
    c = 5
    assert F[c, 0] == pytest.approx(means[0, c] / (abs(means[0, c]) + sig[0]))
    up = s.mesh.neighbor(0, 1)[c]
    assert F[c, 180 + 9 + 4] == pytest.approx((means[4, up] - means[4, c]) / (abs(means[4, c]) + sig[4]))


def test_features_invariants():
    """Properties of the feature map that do not restate it: (1) degree-0
    homogeneity: scaling the state and the scales sigma by the same factor
    leaves every feature unchanged; (2) a state that is constant in space has
    zero neighbour differences and zero higher-mode features; (3) shifting the
    periodic state by one cell along an axis permutes the feature rows the
    same way (neighbour features follow their neighbours)."""
    s = dg.DG(dg.Mesh.uniform(3, 4), 3)
    w = s.project(dg.conserved_field(wl.Blast(2000), 5 / 3, 9))
    sig = mlp.feature_scale(s, w)
    F = mlp.features(s, w, sig)
    assert np.allclose(mlp.features(s, 3.7 * w, 3.7 * sig), F, rtol=1e-13, atol=1e-15)
    const = np.zeros_like(w)
    for v in range(9):
        const[:, v * s.n] = 1.0 + v
    Fc = mlp.features(s, const, sig)
    assert np.all(Fc[:, 180:] == 0.0)
    for v in range(9):
        assert np.all(Fc[:, v * 20 + 1:v * 20 + 20] == 0.0)
        assert np.allclose(Fc[:, v * 20], (1.0 + v) / (1.0 + v + sig[v]))
    for a in range(3):
        up = s.mesh.neighbor(a, 1)          # cell c+1 along a
        shifted = w[up]                     # shifted[c] = w[c+1]
        assert np.allclose(mlp.features(s, shifted, sig), F[up], rtol=0, atol=0)
