"""Pins of the oracle's pointwise physics: flux definition, HLLD properties,
GLM upwinding (no GPU)."""
import numpy as np
import pytest

from oracle import physics as ph

G = 5.0 / 3.0


def random_states(rng, n, glm=True):
    rho = rng.uniform(0.5, 2.0, n)
    v = rng.uniform(-1.0, 1.0, (3, n))
    p = rng.uniform(0.2, 2.0, n)
    B = rng.uniform(-1.5, 1.5, (3, n))
    psi = rng.uniform(-0.5, 0.5, n) if glm else None
    return ph.prim_to_cons(rho, v, p, B, G, psi)


def test_flux_matches_tensor_form():
    # eq. mhd-flux written as a matrix: columns of [rho v; rho v v^T + pT I - B B^T;
    # (E+pT) v - (v.B) B; B v^T - v B^T]
    rng = np.random.default_rng(1)
    U = random_states(rng, 20, glm=False)
    for k in range(20):
        u = U[:, k]
        rho, v, E, Bv = u[0], u[1:4] / u[0], u[4], u[5:8]
        p = (G - 1) * (E - 0.5 * rho * v @ v - 0.5 * Bv @ Bv)
        pt = p + 0.5 * Bv @ Bv
        T = np.zeros((8, 3))
        T[0] = rho * v
        T[1:4] = rho * np.outer(v, v) + pt * np.eye(3) - np.outer(Bv, Bv)
        T[4] = (E + pt) * v - (v @ Bv) * Bv
        T[5:8] = np.outer(Bv, v) - np.outer(v, Bv)
        for a in range(3):
            assert np.allclose(ph.flux(u[:, None], a, G)[:, 0], T[:, a], atol=1e-14, rtol=1e-13)
            assert ph.flux(u[:, None], a, G)[5 + a, 0] == 0.0  # no normal-B flux


@pytest.mark.parametrize("glm", [False, True])
def test_numerical_flux_consistency(glm):
    rng = np.random.default_rng(2)
    U = random_states(rng, 200, glm=glm)
    for a in range(3):
        F, bnF = ph.numerical_flux(U, U, a, G, glm=glm, ch=2.5)
        Fa = ph.flux(U, a, G, glm=glm, ch=2.5)
        assert np.allclose(F, Fa, atol=1e-13, rtol=1e-12)
        assert np.allclose(bnF, U[5 + a], rtol=1e-15)


def test_hlld_upwind_branches():
    rng = np.random.default_rng(3)
    UL = random_states(rng, 100, glm=False)
    UR = random_states(rng, 100, glm=False)
    # super-fast flow to the right: F = F_L (with the common face normal field)
    for sgn in (+1, -1):
        A, Bs = UL.copy(), UR.copy()
        for U in (A, Bs):
            rho = U[0]
            v = U[1:4] / rho
            p = ph.pressure(U, G)
            v[0] += sgn * 30.0
            U[:] = ph.prim_to_cons(rho, v, p, U[5:8], G)
        F, bnF = ph.numerical_flux(A, Bs, 0, G)
        up = A if sgn > 0 else Bs
        rho = up[0]
        v = up[1:4] / rho
        p = ph.pressure(up, G)
        Bv = up[5:8].copy()
        Bv[0] = bnF
        Uup = ph.prim_to_cons(rho, v, p, Bv, G)
        assert np.allclose(F, ph.flux(Uup, 0, G), rtol=1e-13, atol=1e-12)


def test_hlld_stationary_contact():
    # v = 0, equal p and B, density jump: no mass or energy flux, momentum = pT - Bn^2
    n = 50
    rng = np.random.default_rng(4)
    Bv = rng.uniform(-1, 1, (3, n))
    p = rng.uniform(0.5, 2, n)
    z = np.zeros((3, n))
    UL = ph.prim_to_cons(rng.uniform(0.5, 1, n), z, p, Bv, G)
    UR = ph.prim_to_cons(rng.uniform(1, 3, n), z, p, Bv, G)
    F, _ = ph.numerical_flux(UL, UR, 0, G)
    assert np.abs(F[0]).max() < 1e-14
    assert np.abs(F[4]).max() < 1e-13
    assert np.allclose(F[1], p + 0.5 * (Bv ** 2).sum(0) - Bv[0] ** 2, rtol=1e-13)
    assert np.abs(F[5:8]).max() < 1e-13


def test_hlld_mirror_symmetry():
    # reflecting x -> -x swaps L/R and flips normal velocity and normal field;
    # the flux of even components flips sign, odd ones keep it
    rng = np.random.default_rng(5)
    UL = random_states(rng, 100, glm=False)
    UR = random_states(rng, 100, glm=False)
    M = np.ones(8)
    M[1] = -1.0
    M[5] = -1.0
    F, _ = ph.numerical_flux(UL, UR, 0, G)
    Fm, _ = ph.numerical_flux(UR * M[:, None], UL * M[:, None], 0, G)
    assert np.allclose(Fm, -(F * M[:, None]), rtol=1e-12, atol=1e-12)


def test_hlld_axis_permutation():
    rng = np.random.default_rng(6)
    UL = random_states(rng, 100, glm=True)
    UR = random_states(rng, 100, glm=True)
    perm = lambda U, s: np.concatenate([U[:1], np.roll(U[1:4], s, 0), U[4:5], np.roll(U[5:8], s, 0), U[8:]])
    F0, _ = ph.numerical_flux(UL, UR, 0, G, glm=True, ch=3.0)
    for a in (1, 2):
        Fa, _ = ph.numerical_flux(perm(UL, a), perm(UR, a), a, G, glm=True, ch=3.0)
        assert np.allclose(Fa, perm(F0, a), rtol=1e-13, atol=1e-13)


def _hllc_toro(UL, UR):
    """HLLC of Toro with the star energy (E/rho + (S*-u)(S* + p/(rho (S-u)))),
    for B = 0; wave speeds +-max fast speed as in the HLLD estimate."""
    def prim(U):
        rho = U[0]
        u = U[1] / rho
        p = ph.pressure(U, G)
        return rho, u, p, np.sqrt(G * p / rho)
    rL, uL, pL, cL = prim(UL)
    rR, uR, pR, cR = prim(UR)
    c = np.maximum(cL, cR)
    SL, SR = np.minimum(uL, uR) - c, np.maximum(uL, uR) + c
    Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR))
    def star(U, r, u, p, S):
        f = r * (S - u) / (S - Ss)
        return np.stack([f, f * Ss, f * U[2] / r, f * U[3] / r,
                         f * (U[4] / r + (Ss - u) * (Ss + p / (r * (S - u)))), 0 * f, 0 * f, 0 * f])
    FL, FR = ph.flux(UL, 0, G), ph.flux(UR, 0, G)
    FsL = FL + SL * (star(UL, rL, uL, pL, SL) - UL)
    FsR = FR + SR * (star(UR, rR, uR, pR, SR) - UR)
    return np.where(SL > 0, FL, np.where(Ss > 0, FsL, np.where(SR > 0, FsR, FR)))


def test_hlld_reduces_to_hllc_without_field():
    rng = np.random.default_rng(7)
    n = 300
    mk = lambda: ph.prim_to_cons(rng.uniform(0.2, 3, n), rng.uniform(-2, 2, (3, n)),
                                 rng.uniform(0.1, 3, n), np.zeros((3, n)), G)
    UL, UR = mk(), mk()
    F, _ = ph.numerical_flux(UL, UR, 0, G)
    assert np.allclose(F, _hllc_toro(UL, UR), rtol=1e-12, atol=1e-12)


def test_glm_upwind_exact_for_linear_waves():
    # For the linear GLM subsystem, (Bn*, psi*) is the exact Riemann state:
    # its characteristic variables psi +- ch Bn are taken from the upwind sides.
    rng = np.random.default_rng(8)
    ch = 1.7
    UL = random_states(rng, 50)
    UR = random_states(rng, 50)
    F, _ = ph.numerical_flux(UL, UR, 0, G, glm=True, ch=ch)
    psi_s, bn_s = F[5], F[8] / ch ** 2
    # w+ = psi + ch Bn travels right (from L), w- = psi - ch Bn travels left (from R)
    assert np.allclose(psi_s + ch * bn_s, UL[8] + ch * UL[5], rtol=1e-13)
    assert np.allclose(psi_s - ch * bn_s, UR[8] - ch * UR[5], rtol=1e-13)


def test_face_normal_field_alfven_weighting():
    # eq. bxface-average-alfven: equal densities -> arithmetic mean; lies between the two
    rng = np.random.default_rng(9)
    bl, br = rng.normal(size=100), rng.normal(size=100)
    rl, rr = rng.uniform(0.1, 5, 100), rng.uniform(0.1, 5, 100)
    assert np.allclose(ph.face_normal_field(bl, rl, br, rl), 0.5 * (bl + br))
    b = ph.face_normal_field(bl, rl, br, rr)
    assert np.all((b - np.minimum(bl, br) > -1e-15) & (np.maximum(bl, br) - b > -1e-15))
    # the lighter side (larger Alfven speed) gets the larger weight
    b = ph.face_normal_field(np.array([1.0]), np.array([0.25]), np.array([0.0]), np.array([4.0]))
    assert np.isclose(b[0], 0.8)


@pytest.mark.parametrize("wave", [-1, +1])
@pytest.mark.parametrize("speed", [0.07, -0.05])
@pytest.mark.parametrize("bn", [0.8, -0.6])
def test_hlld_resolves_isolated_rotational_discontinuity(wave, speed, bn):
    """An isolated rotational (Alfven) discontinuity is resolved exactly by
    HLLD (its middle waves are the Alfven waves): rho, p, u_n, B_n and |B_t|
    are continuous, B_t rotates and v_t jumps by -wave sgn(B_n) [B_t]/sqrt(rho)
    where the discontinuity moves at u_n + wave |B_n|/sqrt(rho) (the jump
    conditions of the ideal-MHD system in the discontinuity's frame).  The
    exact face flux is that of the state on the face: F(U_L) if the
    discontinuity moves right, F(U_R) if it moves left."""
    rho, p = 1.3, 0.7
    sq = np.sqrt(rho)
    un = speed - wave * abs(bn) / sq          # the discontinuity moves at `speed`
    btL = np.array([0.5, -0.35])
    th = 1.1
    btR = np.array([np.cos(th) * btL[0] - np.sin(th) * btL[1], np.sin(th) * btL[0] + np.cos(th) * btL[1]])
    vtL = np.array([0.2, -0.1])
    vtR = vtL - wave * np.sign(bn) * (btR - btL) / sq
    UL = ph.prim_to_cons(np.array([rho]), np.array([[un], [vtL[0]], [vtL[1]]]), np.array([p]),
                         np.array([[bn], [btL[0]], [btL[1]]]), G)
    UR = ph.prim_to_cons(np.array([rho]), np.array([[un], [vtR[0]], [vtR[1]]]), np.array([p]),
                         np.array([[bn], [btR[0]], [btR[1]]]), G)
    fL, fR = ph.flux(UL, 0, G)[:, 0], ph.flux(UR, 0, G)[:, 0]
    # the constructed pair satisfies the jump conditions at that speed
    assert np.allclose(fR - fL, speed * (UR - UL)[:, 0], atol=1e-14)
    F, bnF = ph.numerical_flux(UL, UR, 0, G)
    expect = fL if speed > 0 else fR
    assert np.allclose(F[:, 0], expect, rtol=1e-13, atol=1e-13 * np.abs(expect).max())


def test_powell_q_interp_is_the_path_integral_of_q():
    """eq. powellq-interp: q integrated along the straight path in primitive
    variables (v, B) from the trace to the interface state; a 3-point
    Gauss-Legendre rule in the path parameter integrates the quadratic v.B
    exactly."""
    rng = np.random.default_rng(9)
    U = random_states(rng, 30, glm=False)
    vF = rng.uniform(-1, 1, (3, 30))
    BF = rng.uniform(-1, 1, (3, 30))
    q = ph.powell_q_interp(U, vF, BF)
    v = U[1:4] / U[0]
    Bv = U[5:8]
    xs, ws = np.polynomial.legendre.leggauss(3)
    acc = np.zeros_like(q)
    for x, wgt in zip(xs, ws):
        s = 0.5 * (x + 1.0)
        vs = (1 - s) * v + s * vF
        Bs = (1 - s) * Bv + s * BF
        Us = ph.prim_to_cons(np.ones(30), vs, np.ones(30), Bs, G)
        acc += 0.5 * wgt * ph.powell_q(Us)
    assert np.allclose(q, acc, rtol=1e-14, atol=1e-14)
    # no interface jump: q-dagger is q of the trace
    assert np.allclose(ph.powell_q_interp(U, v, Bv), ph.powell_q(U), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("speed", [0.07, -0.05])
def test_hlld_interface_state_of_a_rotational_discontinuity(speed):
    """The fan state on the face: the left state when the isolated rotational
    discontinuity moves right, the right state when it moves left."""
    rho, p, bn = 1.3, 0.7, 0.8
    sq = np.sqrt(rho)
    un = speed + abs(bn) / sq          # left-going Alfven discontinuity moving at `speed`
    btL = np.array([0.5, -0.35])
    th = 1.1
    btR = np.array([np.cos(th) * btL[0] - np.sin(th) * btL[1], np.sin(th) * btL[0] + np.cos(th) * btL[1]])
    vtL = np.array([0.2, -0.1])
    vtR = vtL + np.sign(bn) * (btR - btL) / sq
    UL = ph.prim_to_cons(np.array([rho]), np.array([[un], [vtL[0]], [vtL[1]]]), np.array([p]),
                         np.array([[bn], [btL[0]], [btL[1]]]), G)
    UR = ph.prim_to_cons(np.array([rho]), np.array([[un], [vtR[0]], [vtR[1]]]), np.array([p]),
                         np.array([[bn], [btR[0]], [btR[1]]]), G)
    F, bnF, vF, BF = ph.numerical_flux(UL, UR, 0, G, state=True)
    up = UL if speed > 0 else UR
    assert np.allclose(vF[:, 0], up[1:4, 0] / up[0, 0], atol=1e-13)
    assert np.allclose(BF[:, 0], up[5:8, 0], atol=1e-13)
    # and the flux is that of the interface state
    assert np.allclose(F[:, 0], ph.flux(up, 0, G)[:, 0], atol=1e-13)


def test_hlld_interface_state_limits():
    rng = np.random.default_rng(12)
    U = random_states(rng, 40, glm=False)
    F, bnF, vF, BF = ph.numerical_flux(U, U, 1, G, state=True)
    assert np.allclose(vF, U[1:4] / U[0], rtol=1e-13, atol=1e-14)
    assert np.allclose(BF, U[5:8], rtol=1e-13, atol=1e-14)
    # supersonic flow to the right: the interface state is the left state (B_n set to B^n_F)
    A, Bs = random_states(rng, 40, glm=False), random_states(rng, 40, glm=False)
    for Ux in (A, Bs):
        rho = Ux[0]
        v = Ux[1:4] / rho
        p = ph.pressure(Ux, G)
        v[0] += 30.0
        Ux[:] = ph.prim_to_cons(rho, v, p, Ux[5:8], G)
    F, bnF, vF, BF = ph.numerical_flux(A, Bs, 0, G, state=True)
    assert np.allclose(vF, A[1:4] / A[0], rtol=1e-14)
    assert np.allclose(BF[1:], A[6:8], rtol=1e-14) and np.allclose(BF[0], bnF)
