"""Characteristic matrices of the 1-D ideal-MHD system (oracle; test
infrastructure only), used by the characteristic slope limiter (Sec. 4.2.2).

The paper does not print the eigenvectors; it points to the literature.  This
module derives them from the primitive-variable Jacobian of 1-D MHD along the
normal n with constant B_n, W = (rho, u_n, u_t1, u_t2, p, B_t1, B_t2):

  entropy   lambda = u                 r = (1, 0, 0, 0, 0, 0, 0)
  Alfven    lambda = u -+ c_a          r = (0, 0, -b2, b1, 0, -+ S sqrt(rho) b2, +- S sqrt(rho) b1)
  fast      lambda = u +- c_f          r = (rho af, +- af cf, -+ as cs S b1, -+ as cs S b2,
                                            rho af a^2, as sqrt(rho) a b1, as sqrt(rho) a b2)
  slow      lambda = u +- c_s          r = (rho as, +- as cs, +- af cf S b1, +- af cf S b2,
                                            rho as a^2, -af sqrt(rho) a b1, -af sqrt(rho) a b2)

with a^2 = gamma p / rho, c_a = |B_n|/sqrt(rho), c_f, c_s the fast and slow
speeds, S = sign(B_n) (sign(0) = +1), (b1, b2) the unit tangential field
direction ((1, 1)/sqrt 2 when B_t = 0) and the Roe & Balsara (1996)
normalisation af^2 = (a^2 - c_s^2)/(c_f^2 - c_s^2),
as^2 = (c_f^2 - a^2)/(c_f^2 - c_s^2) (af = 1, as = 0 when c_f = c_s).
Conserved right eigenvectors are dU/dW times these; the left eigenvectors are
the matrix inverse.  Under GLM cleaning the (B_n, psi) pair adds the exact
block r = (1, +- c_h), l = (1, +- 1/c_h)/2 (eigenvalues +- c_h).

Powell scheme (8 waves, Sec. 4.1.3): with the source term the normal field
obeys dB_n/dt + u dB_n/dx = 0 and no other primitive equation contains
dB_n/dx, so in primitive variables B_n is a decoupled advected quantity, the
divergence wave lambda = u.  Its conserved right eigenvector is dU/dW e_{B_n}
= (0, 0, 0, 0, B_n, 1, 0, 0) in the frame order (rho, m_n, m_t1, m_t2, E,
B_n, B_t1, B_t2); the other seven are the 7-wave vectors with B_n component 0.
"""
import numpy as np

from . import physics as ph


def primitive_right_eigenvectors(rho, u, p, bn, bt1, bt2, gamma):
    """7x7 right eigenvectors (columns) in primitive variables and eigenvalues."""
    a2 = gamma * p / rho
    bt2sq = bt1 * bt1 + bt2 * bt2
    ca2 = bn * bn / rho
    tt = bt2sq / rho                       # tangential Alfven term, b^2 = c_a^2 + tt
    b2 = ca2 + tt
    # every quantity below is formed without cancellation, so that states
    # near the degenerate points (B_t -> 0, c_a -> 0) give eigenvectors that
    # are continuous at rounding level, not at the square root of it:
    #   (c_f^2 - c_s^2)^2 = (a^2 - c_a^2)^2 + tt (2 (a^2 + c_a^2) + tt)
    #   c_f^2 c_s^2 = a^2 c_a^2
    #   x = c_f^2 - a^2 and y = a^2 - c_s^2 have x + y = c_f^2 - c_s^2 and
    #   x y = a^2 tt; the larger of the two is a sum of non-negative terms
    dd = np.sqrt((a2 - ca2) ** 2 + tt * (2.0 * (a2 + ca2) + tt))
    cf2 = 0.5 * (a2 + b2 + dd)
    cs2 = a2 * ca2 / cf2
    cf, cs, ca, a = np.sqrt(cf2), np.sqrt(cs2), np.sqrt(ca2), np.sqrt(a2)
    if dd > 1e-12 * cf2:
        if b2 >= a2:
            x = 0.5 * (b2 - a2 + dd)
            y = a2 * tt / x
        else:
            y = 0.5 * (a2 - b2 + dd)
            x = a2 * tt / y
        af = np.sqrt(min(max(y / dd, 0.0), 1.0))
        as_ = np.sqrt(min(max(x / dd, 0.0), 1.0))
    else:
        af, as_ = 1.0, 0.0
    bt = np.sqrt(bt2sq)
    if bt > 1e-12 * np.sqrt(bn * bn + bt2sq + 1e-300):
        b1, b2_ = bt1 / bt, bt2 / bt
    else:
        b1 = b2_ = 1.0 / np.sqrt(2.0)
    S = 1.0 if bn >= 0.0 else -1.0
    sr = np.sqrt(rho)
    R = np.zeros((7, 7))
    lam = np.zeros(7)
    # order: fast-, Alfven-, slow-, entropy, slow+, Alfven+, fast+
    for k, sgn in ((0, -1.0), (6, 1.0)):
        R[:, k] = [rho * af, sgn * af * cf, -sgn * as_ * cs * S * b1, -sgn * as_ * cs * S * b2_,
                   rho * af * a2, as_ * sr * a * b1, as_ * sr * a * b2_]
        lam[k] = u + sgn * cf
    for k, sgn in ((1, -1.0), (5, 1.0)):
        R[:, k] = [0.0, 0.0, -b2_, b1, 0.0, sgn * S * sr * b2_, -sgn * S * sr * b1]
        lam[k] = u + sgn * ca
    for k, sgn in ((2, -1.0), (4, 1.0)):
        R[:, k] = [rho * as_, sgn * as_ * cs, sgn * af * cf * S * b1, sgn * af * cf * S * b2_,
                   rho * as_ * a2, -af * sr * a * b1, -af * sr * a * b2_]
        lam[k] = u + sgn * cs
    R[:, 3] = [1.0, 0, 0, 0, 0, 0, 0]
    lam[3] = u
    return R, lam


def dU_dW(rho, u, v, w, bt1, bt2, gamma):
    """Jacobian of (rho, m_n, m_t1, m_t2, E, B_t1, B_t2) w.r.t. (rho, u, v, w, p, B_t1, B_t2)."""
    J = np.zeros((7, 7))
    J[0, 0] = 1.0
    J[1, 0], J[1, 1] = u, rho
    J[2, 0], J[2, 2] = v, rho
    J[3, 0], J[3, 3] = w, rho
    J[4, :] = [0.5 * (u * u + v * v + w * w), rho * u, rho * v, rho * w, 1.0 / (gamma - 1.0), bt1, bt2]
    J[5, 5] = 1.0
    J[6, 6] = 1.0
    return J


# frame variable order (rho, m_n, m_t1, m_t2, E, B_n, B_t1, B_t2, psi) -> indices of
# the 7-wave block and of the GLM pair
IDX7 = [0, 1, 2, 3, 4, 6, 7]
IDXG = [5, 8]


def frame_permutation(a):
    """Global conserved index of each frame variable for normal axis a."""
    n, t1, t2 = ph.face_frame(a)
    return [ph.RHO, ph.M1 + n, ph.M1 + t1, ph.M1 + t2, ph.EN, ph.B1 + n, ph.B1 + t1, ph.B1 + t2, ph.PSI]


def char_matrices(ubar, a, gamma, ch, nvar=9):
    """(L, R) in global conserved components for normal axis a at the state
    ubar (nvar = 9: 7-wave MHD block + GLM pair; nvar = 8: the Powell 8-wave
    system; L R = I)."""
    perm = frame_permutation(a)[:nvar]
    uf = ubar[perm]
    rho = uf[0]
    u, v, w = uf[1] / rho, uf[2] / rho, uf[3] / rho
    p = ph.pressure(ubar, gamma)
    bn, bt1, bt2 = uf[5], uf[6], uf[7]
    Rw, lam = primitive_right_eigenvectors(rho, u, p, bn, bt1, bt2, gamma)
    R7 = dU_dW(rho, u, v, w, bt1, bt2, gamma) @ Rw
    L7 = np.linalg.inv(R7)
    Rf = np.zeros((nvar, nvar))
    Lf = np.zeros((nvar, nvar))
    Rf[np.ix_(IDX7, IDX7)] = R7
    Lf[np.ix_(IDX7, IDX7)] = L7
    if nvar == 9:
        Rf[np.ix_(IDXG, IDXG)] = [[1.0, 1.0], [ch, -ch]]
        Lf[np.ix_(IDXG, IDXG)] = [[0.5, 0.5 / ch], [0.5, -0.5 / ch]]
    else:
        # Powell divergence wave: r = (0, 0, 0, 0, B_n, 1, 0, 0); L = R^-1 block-wise
        Rf[5, 5] = 1.0
        Rf[4, 5] = bn
        Lf[5, 5] = 1.0
        Lf[IDX7, 5] = -L7[:, 4] * bn
    # back to global component order
    P = np.zeros((nvar, nvar))
    for i, g in enumerate(perm):
        P[g, i] = 1.0
    R = P @ Rf
    L = Lf @ P.T
    return L, R
