"""Slope and positivity limiters (oracle; test infrastructure only).

TVB slope limiter (Sec. 4.2.1, eq. tvb-limiter): per cell and direction, the
slope a (the weight of the degree-1 Legendre mode along that direction) is
compared with the neighbour mean differences Delta = (mean_{i+1} - mean_i)/2
and (mean_i - mean_{i-1})/2; with the threshold M = M~/dx kept at M~ constant,
sigma = a if |a| <= M~ dx, else minmod(a, beta Delta_L, beta Delta_R); the
cell is troubled when |sigma - a| > eps for some direction and variable.
Characteristic limiting (Sec. 4.2.2) applies this to L(mean) . a and maps the
limited slopes back with R.  A troubled cell gets the limited slopes in the
directions that triggered, keeps its other slopes unchanged and loses all
modes of degree >= 2 (all variables).

LDF slope fix (Sec. 4.2.4): diagonal slopes rescaled so that their sum is
zero (delta+- rule), then the linear field is L2-projected on the LDF basis.

Positivity limiter (Sec. 4.3, eq. wtilde, eq. tau_rho, eq. tau_press): floors
on the cell averages (tallied), then w <- tau w + (1 - tau) w_mean with tau
the smallest of (rho_bar - eps)/(rho_bar - rho_q) over points with
rho_q < eps and (p_bar - eps)/(p_bar - p_q) over points with p_q < eps,
over all volume and face quadrature points.  Reading: p_q only counts where
rho_q > 0; a point counts only where it lies below the mean (the ratio is
taken where its denominator is positive) and tau is clipped to [0, 1], so a
cell whose mean sits at the floor collapses to its mean; a second pass is
made if the first one leaves any point below half the floors (rounding at
the floor level after the first pass is not re-limited).
"""
import numpy as np

from . import eigen
from . import physics as ph
from .dg import GLM, POWELL


def minmod(a, b, c):
    out = np.zeros(np.broadcast(a, b, c).shape)
    pos = (a > 0) & (b > 0) & (c > 0)
    neg = (a < 0) & (b < 0) & (c < 0)
    out = np.where(pos, np.minimum(np.minimum(a, b), c), out)
    out = np.where(neg, np.maximum(np.maximum(a, b), c), out)
    return out


def tvb_sigma(a, dl, dr, Mtilde, h, beta):
    """Limited slope of eq. tvb-limiter with M = M~/h."""
    return np.where(np.abs(a) <= Mtilde * h, a, minmod(a, beta * dl, beta * dr))


def char_usable(ubar, gamma, rel=1e-8):
    """Whether the characteristic matrices at the cell mean ubar are used
    (Sec. 4.2.2).  Their condition number grows like b^2/a^2 (Alfven over
    sound speed squared), so near the positivity floor in a strong field the
    projection carries no accurate digit; the paper does not treat this
    case.  Reading: such a cell (gamma p < rel (gamma p + |B|^2), or a
    non-positive density or pressure) is limited componentwise."""
    rho = ubar[ph.RHO]
    gp = gamma * ph.pressure(ubar, gamma)
    B2 = ubar[ph.B1] ** 2 + ubar[ph.B2] ** 2 + ubar[ph.B3] ** 2
    return bool(rho > 0.0 and gp > 0.0 and gp >= rel * (gp + B2))


def slope_limit(s, w, Mtilde=5.0, beta=2.0, eps=1e-8, characteristic=True, ch=1.0):
    """TVB (characteristic) slope limiter on a uniform grid.  GLM: Legendre
    basis, 9 variables.  Powell: the LDF magnetic field (slope_limit_powell).
    Returns (w_new, troubled flags)."""
    if s.divb == POWELL:
        return slope_limit_powell(s, w, Mtilde, beta, eps, characteristic)
    assert s.divb == GLM
    D, n = s.D, s.n
    C = w.shape[0]
    h = s.mesh.h
    means = s.cell_means(w)  # [var, C]
    out = w.copy()
    troubled = np.zeros(C, dtype=bool)
    new_slopes = {}
    for a in range(D):
        up = s.mesh.neighbor(a, +1)
        dn = s.mesh.neighbor(a, -1)
        lslope = 1 + a  # Legendre mode with exponent e_a
        slope = w[:, [v * n + lslope for v in range(9)]].T  # [var, C]
        dl = 0.5 * (means[:, up] - means)
        dr = 0.5 * (means - means[:, dn])
        sig_cons = np.empty_like(slope)
        trig = np.zeros(C, dtype=bool)
        for c in range(C):
            if characteristic and char_usable(means[:, c], s.gamma):
                L, R = eigen.char_matrices(means[:, c], a, s.gamma, ch)
            else:
                L = R = np.eye(9)
            ca, cl, cr = L @ slope[:, c], L @ dl[:, c], L @ dr[:, c]
            sig = tvb_sigma(ca, cl, cr, Mtilde, h[c], beta)
            t = np.abs(sig - ca) > eps
            trig[c] = t.any()
            sig_cons[:, c] = R @ np.where(t, sig, ca)
        new_slopes[a] = (trig, sig_cons)
        troubled |= trig
    for a in range(D):
        trig, sig_cons = new_slopes[a]
        sel = troubled & trig
        for v in range(9):
            out[sel, v * n + 1 + a] = sig_cons[v, sel]
    hi = [v * n + l for v in range(9) for l in range(D + 1, n)]
    out[np.ix_(troubled, hi)] = 0.0
    return out, troubled


def ldf_moments(s):
    """For each LDF function l and component c: its cell average (Pm[c, l])
    and its linear coefficient along xi_b, <Phi_lc, xi_b>/<xi_b, xi_b>
    (Pl[c, b, l]), by the (d+2)-point rule (exact: degree <= d + 1)."""
    from .quadrature import tensor_rule
    xq, wq = tensor_rule(s.d + 2, s.D)
    from . import basis as Bm
    Phi = Bm.ldf_values(s.D, s.d, xq)                      # [c, q, l]
    vol = 2.0 ** s.D
    Pm = np.einsum("q,cql->cl", wq, Phi) / vol
    Pl = np.einsum("q,qb,cql->cbl", wq, xq, Phi) / (vol / 3.0)
    return Pm, Pl


def slope_limit_powell(s, w, Mtilde=5.0, beta=2.0, eps=1e-8, characteristic=True):
    """TVB slope limiter for the Powell scheme (Sec. 4.2.1-4.2.2, 4.2.4).
    Per cell and direction b the 8-component slope (rho, m, E and the linear
    coefficients S[c, b] of the LDF magnetic field) and the neighbour mean
    differences go to the 8-wave characteristic variables (eigen, nvar = 8)
    and are limited as in slope_limit.  A troubled cell: rho, m, E take the
    limited slopes of the triggered directions and lose their modes of degree
    >= 2; the magnetic field becomes the linear field mean + S' xi, S' the
    limited slope matrix with its diagonal made divergence-free by the
    delta+- rescaling (ldf_divfree_fix), L2-projected onto the LDF basis
    (exact: a divergence-free linear field)."""
    D, n = s.D, s.n
    C = w.shape[0]
    h = s.mesh.h
    means = s.cell_means(w)                                 # [8, C]
    nl = len(s.leg_vars) * n
    wb = w[:, nl:]
    Pm, Pl = ldf_moments(s)
    S = np.einsum("cbl,kl->kcb", Pl, wb)                    # [C, c, b] magnetic slopes
    out = w.copy()
    troubled = np.zeros(C, dtype=bool)
    new_slopes = {}
    for a in range(D):
        up = s.mesh.neighbor(a, +1)
        dn = s.mesh.neighbor(a, -1)
        slope = np.zeros((8, C))
        for j, v in enumerate(s.leg_vars):
            slope[v] = w[:, j * n + 1 + a]
        for c in range(D):
            slope[ph.B1 + c] = S[:, c, a]
        dl = 0.5 * (means[:, up] - means)
        dr = 0.5 * (means - means[:, dn])
        sig_cons = np.empty_like(slope)
        trig = np.zeros(C, dtype=bool)
        for k in range(C):
            if characteristic and char_usable(means[:, k], s.gamma):
                L, R = eigen.char_matrices(means[:, k], a, s.gamma, None, nvar=8)
            else:
                L = R = np.eye(8)
            ca, cl, cr = L @ slope[:, k], L @ dl[:, k], L @ dr[:, k]
            sig = tvb_sigma(ca, cl, cr, Mtilde, h[k], beta)
            t = np.abs(sig - ca) > eps
            trig[k] = t.any()
            sig_cons[:, k] = R @ np.where(t, sig, ca)
        new_slopes[a] = (trig, sig_cons)
        troubled |= trig
    for a in range(D):
        trig, sig_cons = new_slopes[a]
        sel = troubled & trig
        for j, v in enumerate(s.leg_vars):
            out[sel, j * n + 1 + a] = sig_cons[v, sel]
        for c in range(D):
            S[sel, c, a] = sig_cons[ph.B1 + c, sel]
    hi = [j * n + l for j in range(len(s.leg_vars)) for l in range(D + 1, n)]
    out[np.ix_(troubled, hi)] = 0.0
    for k in np.nonzero(troubled)[0]:
        Sk = ldf_divfree_fix(S[k])
        out[k, nl:] = ldf_project_linear(s, means[ph.B1:ph.B1 + D, k], Sk)
    return out, troubled


def ldf_divfree_fix(S):
    """delta+- rescaling of Sec. 4.2.4 on a slope matrix S[c, b] = dB_c/dxi_b:
    returns S with corrected diagonal (sum zero, |sigma~| <= |sigma|)."""
    S = np.array(S, dtype=np.float64)
    D = S.shape[0]
    sig = np.diag(S).copy()
    dp = np.maximum(sig, 0.0).sum()
    dm = np.maximum(-sig, 0.0).sum()
    delta = dp - dm
    if delta > 0:
        sig = np.where(sig > 0, sig * (dm / dp), sig)
    elif delta < 0:
        sig = np.where(sig < 0, sig * (dp / dm), sig)
    for c in range(D):
        S[c, c] = sig[c]
    return S


def ldf_project_linear(s, Bmean, S):
    """LDF weights of the linear field B_c = Bmean_c + sum_b S[c, b] xi_b
    (divergence-free) by L2 projection onto the LDF basis."""
    from .quadrature import tensor_rule
    xq, wq = tensor_rule(s.d + 1, s.D)
    Bq = Bmean[:, None] + S @ xq.T  # [c, q]
    return np.einsum("cq,cql,q->l", Bq, s.Phi, wq) / s.Mldf


def positivity(s, w, eps_rho=1e-12, eps_p=1e-12):
    """Positivity limiter on all volume and face points.  Returns
    (w_new, stats dict)."""
    g = s.gamma
    out = w.copy()
    C = w.shape[0]
    vol = s.mesh.h ** s.D
    stats = dict(n_floor=0, n_pos_scaled=0, injected_mass=0.0, injected_energy=0.0)
    n = s.n
    eidx = s.leg_vars.index(ph.EN) * n
    # floors on the cell averages
    Ub = s.cell_means(out)
    low = Ub[ph.RHO] < eps_rho
    if low.any():
        stats["injected_mass"] += float(((eps_rho - Ub[ph.RHO][low]) * vol[low]).sum())
        out[low, 0] = eps_rho
        stats["n_floor"] += int(low.sum())
        Ub = s.cell_means(out)
    pb = ph.pressure(Ub, g)
    lowp = pb < eps_p
    if lowp.any():
        ke = 0.5 * (Ub[ph.M1] ** 2 + Ub[ph.M2] ** 2 + Ub[ph.M3] ** 2) / Ub[ph.RHO]
        me = 0.5 * (Ub[ph.B1] ** 2 + Ub[ph.B2] ** 2 + Ub[ph.B3] ** 2)
        Enew = eps_p / (g - 1.0) + ke + me
        stats["injected_energy"] += float(((Enew - Ub[ph.EN])[lowp] * vol[lowp]).sum())
        out[lowp, eidx] = Enew[lowp]
        stats["n_floor"] += int(lowp.sum())
        Ub = s.cell_means(out)
        pb = ph.pressure(Ub, g)
    # modes that carry the cell mean (kept by the scaling)
    keep = np.zeros(s.nmodes, dtype=bool)
    keep[[j * n for j in range(len(s.leg_vars))]] = True
    if s.nldf:
        from . import basis as Bm
        degs = Bm.ldf_degrees(s.D, s.d)
        o = len(s.leg_vars) * n
        for l, dgl in enumerate(degs):
            if dgl == 0:
                keep[o + l] = True
    for npass in range(2):
        pts = np.concatenate(s.all_point_states(out), axis=2)  # [var, C, P]
        rq = pts[ph.RHO]
        with np.errstate(divide="ignore", invalid="ignore"):
            pq = ph.pressure(pts, g)
        tau = np.ones(C)
        rb = Ub[ph.RHO][:, None]
        # the second pass acts on points below half the floors only: after the
        # first pass, values at the floor carry rounding from the cancellation
        # in E - m^2/(2 rho) - B^2/2 and must not decide anything
        f = 1.0 if npass == 0 else 0.5
        m = rq < eps_rho * f
        # a point counts only where it lies below the mean (scaling toward the
        # mean cannot raise a point that is not); tau is clipped to [0, 1], so
        # a cell whose mean pressure sits at the floor collapses to its mean
        tr = point_tau(rb, rq, eps_rho, m)
        tp = point_tau(pb[:, None], pq, eps_p, (rq > 0) & (pq < eps_p * f))
        tau = np.clip(np.minimum(tau, np.minimum(tr.min(axis=1), tp.min(axis=1))), 0.0, 1.0)
        sel = tau < 1.0
        if not sel.any():
            break
        stats["n_pos_scaled"] += int(sel.sum())
        out[np.ix_(sel, ~keep)] *= tau[sel][:, None]
    return out, stats


def point_tau(mean, q, floor, mask):
    """Per-point factor of eq. tau_rho / eq. tau_press: (mean - floor) /
    (mean - q) at the masked points that lie below the mean, 1 elsewhere (a
    point not below the mean cannot be raised by scaling toward it)."""
    d = mean - q
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(mask & (d > 0), (mean - floor) / np.where(d > 0, d, 1.0), 1.0)


def make_stage_limiter(s, limiter, Mtilde=5.0, beta=2.0, eps=1e-8, eps_rho=1e-12, eps_p=1e-12, stats=None):
    """Limiter applied after every RK stage: slope limiter, then positivity.
    limiter: bit flags 1 = TVB, 2 = characteristic variables, 4 = positivity.
    Called as lim(w, ch) with the step's c_h (GLM block of the eigensystem);
    ch = None takes c_h from the time-step rule applied to w itself."""
    def lim(w, ch=None):
        if ch is None:
            ch = s.timestep(w)[1] if s.divb == GLM else 0.0
        if limiter & 1:
            w, tr = slope_limit(s, w, Mtilde, beta, eps, characteristic=bool(limiter & 2), ch=ch)
            if stats is not None:
                stats["n_tvb"] = stats.get("n_tvb", 0) + int(tr.sum())
        if limiter & 4:
            w, st = positivity(s, w, eps_rho, eps_p)
            if stats is not None:
                for k, v in st.items():
                    stats[k] = stats.get(k, 0) + v
        return w
    return lim
