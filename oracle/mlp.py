"""Learned troubled-cell indicator (oracle; test infrastructure only).

The paper's limiting is detect-then-limit, with the detector judged by its
sensitivity and specificity (Sec. 4.2).  The build adds a small network that
predicts where the plain TVB detector fires, so that the characteristic
decomposition only runs where it is needed.  This module is its reference:

  features (256): for each of the 9 variables v, the 20 modal weights of the
  cell divided by s_v = |w_mean_v| + sigma_v, then for each of the 6 face
  neighbours the difference of its mean and the cell mean divided by s_v
  (180 + 54 = 234), zero padded to 256; sigma_v is the RMS of the cell means
  of variable v over the initial state, floored at 1e-2 of the largest RMS;
  network: 256 -> 64 -> 64 -> 64 -> 1, GELU (erf form) on the hidden layers,
  sigmoid output, binary cross-entropy loss.

Arithmetic: FP64 (with finite-difference pins), or `bf16=True`, which rounds
to bfloat16 exactly where the GPU kernels feed their BF16 matrix products
(inputs, weights, hidden activations, back-propagated gradients) and keeps
FP32-representable accumulation in float64 otherwise.
"""
import math

import numpy as np

LAYERS = [(256, 64), (64, 64), (64, 64), (64, 1)]
NFEAT = 256


def bf16_round(x):
    """Round float values to bfloat16 (round to nearest even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + _erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def _erf(x):
    from scipy.special import erf
    return erf(x)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def init_params(seed):
    """Weights W[in, out] ~ U(-1/sqrt(in), 1/sqrt(in)), biases zero."""
    rng = np.random.default_rng(seed)
    P = []
    for fin, fout in LAYERS:
        lim = 1.0 / math.sqrt(fin)
        P.append(rng.uniform(-lim, lim, (fin, fout)))
        P.append(np.zeros(fout))
    return P


def forward(P, X, bf16=False):
    """Returns (p, cache).  X [B, 256]."""
    rd = bf16_round if bf16 else (lambda a: a)
    a = rd(X)
    cache = []
    for li in range(4):
        W, b = P[2 * li], P[2 * li + 1]
        z = a @ rd(W) + b
        cache.append((a, z))
        if li < 3:
            a = rd(gelu(z))
    p = sigmoid(z[:, 0])
    return p, cache


def bce(p, y):
    eps = 1e-12
    return float(-np.mean(y * np.log(np.maximum(p, eps)) + (1 - y) * np.log(np.maximum(1 - p, eps))))


def backward(P, X, y, bf16=False):
    """(loss, grads) of the mean BCE loss; grads in the layout of P."""
    rd = bf16_round if bf16 else (lambda a: a)
    p, cache = forward(P, X, bf16)
    B = X.shape[0]
    dz = ((p - y) / B)[:, None]
    grads = [None] * 8
    for li in range(3, -1, -1):
        a, z = cache[li]
        W = P[2 * li]
        dzr = rd(dz)
        grads[2 * li] = a.T @ dzr
        grads[2 * li + 1] = dz.sum(axis=0)
        if li > 0:
            da = dzr @ rd(W).T
            dz = da * gelu_grad(cache[li - 1][1])
    return bce(p, y), grads


def adam_update(P, G, M, V, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) in place; t counts from 1."""
    for i in range(len(P)):
        M[i] = b1 * M[i] + (1 - b1) * G[i]
        V[i] = b2 * V[i] + (1 - b2) * G[i] ** 2
        mh = M[i] / (1 - b1 ** t)
        vh = V[i] / (1 - b2 ** t)
        P[i] = P[i] - lr * mh / (np.sqrt(vh) + eps)


def feature_scale(s, w):
    """sigma_v: RMS over cells of the cell means of each variable, floored at
    1e-2 of the largest of them (a variable that is zero everywhere at t = 0,
    such as the momentum of a state at rest, must not divide by zero)."""
    means = s.cell_means(w)
    rms = np.sqrt((means ** 2).mean(axis=1))
    return np.maximum(rms, 1e-2 * rms.max())


def features(s, w, sigma):
    """Feature matrix [C, 256] of a uniform-grid GLM state (degree 3 has 20
    modes per variable; lower degrees pad the modal block with zeros)."""
    C = w.shape[0]
    n = s.n
    means = s.cell_means(w)  # [9, C]
    scale = np.abs(means) + sigma[:, None]
    F = np.zeros((C, NFEAT))
    for v in range(9):
        F[:, v * 20:v * 20 + n] = w[:, v * n:(v + 1) * n] / scale[v][:, None]
    k = 180
    for a in range(s.D):
        for sgn in (-1, 1):
            nb = s.mesh.neighbor(a, sgn)
            for v in range(9):
                F[:, k] = (means[v, nb] - means[v]) / scale[v]
                k += 1
    return F
