"""Pointwise ideal-MHD physics (oracle; test infrastructure only).

Arrays carry the conserved components on axis 0 and any batch shape behind:
U = (rho, m1, m2, m3, E, B1, B2, B3[, psi]).  Heaviside-Lorentz units
(no 4 pi), ideal gas with adiabatic index gamma (Sec. 2, eq. cns-vec,
eq. mhd-flux).

Face flux (Sec. 4.1.2 "Choice of numerical flux function", Sec. 4.1.3,
Sec. 4.1.5): the face normal field is the Alfven-velocity-weighted average
(eq. bxface-average-alfven); both states keep their thermal pressure and take
that common normal field; the HLLD solver of Miyoshi & Kusano (2005) gives
the flux.  Under GLM cleaning the normal-B and psi fluxes are replaced by the
upwinded linear GLM fluxes psi* and c_h^2 Bn* of Dedner et al. (2002).
"""
import numpy as np

RHO, M1, M2, M3, EN, B1, B2, B3, PSI = range(9)


def pressure(U, gamma):
    """p = (gamma-1)(E - |m|^2/(2 rho) - |B|^2/2)  (eq. cns-vec)."""
    rho = U[RHO]
    ke = 0.5 * (U[M1] ** 2 + U[M2] ** 2 + U[M3] ** 2) / rho
    me = 0.5 * (U[B1] ** 2 + U[B2] ** 2 + U[B3] ** 2)
    return (gamma - 1.0) * (U[EN] - ke - me)


def prim_to_cons(rho, v, p, B, gamma, psi=None):
    """(rho, v[3], p, B[3]) -> U.  E = p/(gamma-1) + rho v^2/2 + B^2/2."""
    E = p / (gamma - 1.0) + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) + 0.5 * (B[0] ** 2 + B[1] ** 2 + B[2] ** 2)
    comps = [rho, rho * v[0], rho * v[1], rho * v[2], E, B[0], B[1], B[2]]
    if psi is not None:
        comps.append(psi)
    return np.stack([np.broadcast_to(np.asarray(c, dtype=np.float64), np.shape(rho)) for c in comps])


def flux(U, a, gamma, glm=False, ch=0.0):
    """Analytic flux f_a(U) along axis a (eq. mhd-flux); GLM adds psi to the
    B_a flux and c_h^2 B_a as the psi flux (Sec. 4.1.5)."""
    rho = U[RHO]
    v = [U[M1] / rho, U[M2] / rho, U[M3] / rho]
    B = [U[B1], U[B2], U[B3]]
    p = pressure(U, gamma)
    pt = p + 0.5 * (B[0] ** 2 + B[1] ** 2 + B[2] ** 2)
    vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2]
    F = np.empty_like(U)
    F[RHO] = rho * v[a]
    for b in range(3):
        F[M1 + b] = rho * v[b] * v[a] - B[b] * B[a]
        F[B1 + b] = B[b] * v[a] - v[b] * B[a]
    F[M1 + a] += pt
    F[EN] = (U[EN] + pt) * v[a] - vB * B[a]
    if glm:
        F[B1 + a] += U[PSI]
        F[PSI] = ch * ch * B[a]
    return F


def signal_speed_sum(U, gamma, D):
    """sum_a (|v_a| + c) with c = sqrt(c_s^2 + c_A^2) (Sec. 3.6, eq. cfl).

    Reading for states that the positivity limiter has not yet seen (an
    unlimited initial projection): the sound speed uses max(p, 0) and points
    with rho <= 0 do not contribute."""
    rho = U[RHO]
    ok = rho > 0.0
    rs = np.where(ok, rho, 1.0)
    p = np.maximum(pressure(np.where(ok, U, 1.0), gamma), 0.0)
    bsq = U[B1] ** 2 + U[B2] ** 2 + U[B3] ** 2
    c = np.sqrt((gamma * p + bsq) / rs)
    s = np.zeros_like(rho)
    for a in range(D):
        s = s + np.abs(U[M1 + a] / rs) + c
    return np.where(ok, s, 0.0)


def face_normal_field(bnL, rhoL, bnR, rhoR):
    """B^n_F weighted by inverse sqrt densities (eq. bxface-average-alfven)."""
    iL = 1.0 / np.sqrt(rhoL)
    iR = 1.0 / np.sqrt(rhoR)
    return (bnL * iL + bnR * iR) / (iL + iR)


def _sgn(x):
    return np.where(x >= 0.0, 1.0, -1.0)


def hlld(WL, WR, bx, gamma, state=False):
    """HLLD flux of Miyoshi & Kusano (2005) in the face frame.

    WL, WR: primitive states (rho, u, v, w, p, By, Bz) on axis 0; bx the common
    normal field.  Returns the 8-component flux of (rho, m_n, m_t1, m_t2, E,
    B_n, B_t1, B_t2), the B_n component being zero.  state=True also returns
    the state of the fan region that contains the face (x/t = 0) as
    (rho, u, v, w, By, Bz): the interface state of Sec. 4.1.3 ("Interface
    state U_F")."""
    g = gamma

    def cons_and_flux(W):
        rho, u, v, w, p, by, bz = W
        bsq = bx * bx + by * by + bz * bz
        E = p / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w) + 0.5 * bsq
        pt = p + 0.5 * bsq
        vb = u * bx + v * by + w * bz
        U = np.stack([rho, rho * u, rho * v, rho * w, E, np.broadcast_to(bx, rho.shape), by, bz])
        F = np.stack([
            rho * u,
            rho * u * u + pt - bx * bx,
            rho * v * u - bx * by,
            rho * w * u - bx * bz,
            (E + pt) * u - vb * bx,
            np.zeros_like(rho),
            by * u - v * bx,
            bz * u - w * bx,
        ])
        gp = g * p
        disc = np.maximum(((gp + bsq) / rho) ** 2 - 4.0 * gp * bx * bx / (rho * rho), 0.0)
        cf2 = 0.5 * ((gp + bsq) / rho + np.sqrt(disc))
        return U, F, E, pt, np.sqrt(cf2)

    UL, FL, EL, ptL, cfL = cons_and_flux(WL)
    UR, FR, ER, ptR, cfR = cons_and_flux(WR)
    rL, uL, vL, wL, pL, byL, bzL = WL
    rR, uR, vR, wR, pR, byR, bzR = WR

    cmax = np.maximum(cfL, cfR)
    SL = np.minimum(uL, uR) - cmax
    SR = np.maximum(uL, uR) + cmax
    dL = (SL - uL) * rL
    dR = (SR - uR) * rR
    den = dR - dL
    SM = (dR * uR - dL * uL - ptR + ptL) / den
    ptS = (dR * ptL - dL * ptR + rL * rR * (SR - uR) * (SL - uL) * (uR - uL)) / den

    def star(W, U, E, pt, S, d):
        rho, u, v, w, p, by, bz = W
        rs = d / (S - SM)
        dd = d * (S - SM) - bx * bx
        degen = np.abs(dd) <= 1e-12 * np.maximum(rho * (S - u) ** 2, bx * bx)
        safe = np.where(degen, 1.0, dd)
        vs = np.where(degen, v, v - bx * by * (SM - u) / safe)
        ws = np.where(degen, w, w - bx * bz * (SM - u) / safe)
        bys = np.where(degen, by, by * (d * (S - u) - bx * bx) / safe)
        bzs = np.where(degen, bz, bz * (d * (S - u) - bx * bx) / safe)
        vb = u * bx + v * by + w * bz
        vbs = SM * bx + vs * bys + ws * bzs
        Es = ((S - u) * E - pt * u + ptS * SM + bx * (vb - vbs)) / (S - SM)
        Us = np.stack([rs, rs * SM, rs * vs, rs * ws, Es, np.broadcast_to(bx, rho.shape), bys, bzs])
        return Us, rs, vs, ws, bys, bzs, Es, vbs

    UsL, rsL, vsL, wsL, bysL, bzsL, EsL, vbsL = star(WL, UL, EL, ptL, SL, dL)
    UsR, rsR, vsR, wsR, bysR, bzsR, EsR, vbsR = star(WR, UR, ER, ptR, SR, dR)

    sqL = np.sqrt(rsL)
    sqR = np.sqrt(rsR)
    SsL = SM - np.abs(bx) / sqL
    SsR = SM + np.abs(bx) / sqR
    s = _sgn(bx)
    isum = 1.0 / (sqL + sqR)
    vss = (sqL * vsL + sqR * vsR + (bysR - bysL) * s) * isum
    wss = (sqL * wsL + sqR * wsR + (bzsR - bzsL) * s) * isum
    byss = (sqL * bysR + sqR * bysL + sqL * sqR * (vsR - vsL) * s) * isum
    bzss = (sqL * bzsR + sqR * bzsL + sqL * sqR * (wsR - wsL) * s) * isum
    vbss = SM * bx + vss * byss + wss * bzss
    EssL = EsL - sqL * (vbsL - vbss) * s
    EssR = EsR + sqR * (vbsR - vbss) * s
    bxa = np.broadcast_to(bx, rsL.shape)
    UssL = np.stack([rsL, rsL * SM, rsL * vss, rsL * wss, EssL, bxa, byss, bzss])
    UssR = np.stack([rsR, rsR * SM, rsR * vss, rsR * wss, EssR, bxa, byss, bzss])

    FsL = FL + SL * (UsL - UL)
    FsR = FR + SR * (UsR - UR)
    FssL = FsL + SsL * (UssL - UsL)
    FssR = FsR + SsR * (UssR - UsR)

    out = np.where(SL > 0.0, FL,
          np.where(SsL > 0.0, FsL,
          np.where(SM > 0.0, FssL,
          np.where(SsR > 0.0, FssR,
          np.where(SR > 0.0, FsR, FR)))))
    if not state:
        return out
    # the same fan regions, as primitive states
    SMa = np.broadcast_to(SM, rsL.shape)
    stL = np.stack([rL, uL, vL, wL, byL, bzL])
    stR = np.stack([rR, uR, vR, wR, byR, bzR])
    stsL = np.stack([rsL, SMa, vsL, wsL, bysL, bzsL])
    stsR = np.stack([rsR, SMa, vsR, wsR, bysR, bzsR])
    stssL = np.stack([rsL, SMa, vss, wss, byss, bzss])
    stssR = np.stack([rsR, SMa, vss, wss, byss, bzss])
    st = np.where(SL > 0.0, stL,
         np.where(SsL > 0.0, stsL,
         np.where(SM > 0.0, stssL,
         np.where(SsR > 0.0, stssR,
         np.where(SR > 0.0, stsR, stR)))))
    return out, st


def face_frame(a):
    """(normal, tangential 1, tangential 2) axes: a cyclic permutation."""
    return a, (a + 1) % 3, (a + 2) % 3


def numerical_flux(UL, UR, a, gamma, glm=False, ch=0.0, state=False):
    """Numerical flux through a face with normal +e_a (global components).

    Returns (F, bnF): F has the components of U; bnF is the face normal field
    B^n_F (also needed by the Powell face term and the divergence norm).
    state=True returns (F, bnF, vF, BF) with the velocity and magnetic field
    of the HLLD interface state in global components (its normal field is
    B^n_F)."""
    n, t1, t2 = face_frame(a)

    def prim(U):
        rho = U[RHO]
        p = pressure(U, gamma)
        return rho, U[M1 + n] / rho, U[M1 + t1] / rho, U[M1 + t2] / rho, p, U[B1 + t1], U[B1 + t2]

    WL = np.stack(prim(UL))
    WR = np.stack(prim(UR))
    bnL, bnR = UL[B1 + n], UR[B1 + n]
    bnF = face_normal_field(bnL, UL[RHO], bnR, UR[RHO])
    if state:
        Fn, st = hlld(WL, WR, bnF, gamma, state=True)
    else:
        Fn = hlld(WL, WR, bnF, gamma)
    F = np.zeros_like(UL)
    F[RHO] = Fn[0]
    F[M1 + n], F[M1 + t1], F[M1 + t2] = Fn[1], Fn[2], Fn[3]
    F[EN] = Fn[4]
    F[B1 + n], F[B1 + t1], F[B1 + t2] = Fn[5], Fn[6], Fn[7]
    if glm:
        psiL, psiR = UL[PSI], UR[PSI]
        bn_star = 0.5 * (bnL + bnR) - (psiR - psiL) / (2.0 * ch)
        psi_star = 0.5 * (psiL + psiR) - 0.5 * ch * (bnR - bnL)
        F[B1 + n] = psi_star
        F[PSI] = ch * ch * bn_star
    if not state:
        return F, bnF
    vF = np.empty((3,) + np.shape(bnF))
    BF = np.empty((3,) + np.shape(bnF))
    vF[n], vF[t1], vF[t2] = st[1], st[2], st[3]
    BF[n], BF[t1], BF[t2] = bnF, st[4], st[5]
    return F, bnF, vF, BF


def powell_q_interp(U, vF, BF):
    """q-dagger of eq. powellq-interp for a side whose trace is U (conserved)
    and the interface velocity vF and field BF:
    (0, (B + B_F)/2, (2 B.v + B.v_F + B_F.v + 2 B_F.v_F)/6, (v + v_F)/2)."""
    rho = U[RHO]
    v = np.stack([U[M1] / rho, U[M2] / rho, U[M3] / rho])
    B = np.stack([U[B1], U[B2], U[B3]])
    dot = lambda x, y: (x * y).sum(axis=0)
    e = (2.0 * dot(B, v) + dot(B, vF) + dot(BF, v) + 2.0 * dot(BF, vF)) / 6.0
    return np.stack([np.zeros_like(rho), 0.5 * (B[0] + BF[0]), 0.5 * (B[1] + BF[1]), 0.5 * (B[2] + BF[2]), e,
                     0.5 * (v[0] + vF[0]), 0.5 * (v[1] + vF[1]), 0.5 * (v[2] + vF[2])])


def powell_q(U):
    """q(U) = (0, B, v.B, v) over the 8 MHD components (eq. powell-q)."""
    rho = U[RHO]
    v = [U[M1] / rho, U[M2] / rho, U[M3] / rho]
    B = [U[B1], U[B2], U[B3]]
    vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2]
    return np.stack([np.zeros_like(rho), B[0], B[1], B[2], vB, v[0], v[1], v[2]])
