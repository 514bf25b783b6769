"""Modal DG right-hand side, time step and SSP-RK3 (oracle; test infrastructure only).

Weak form (Sec. 3.5, eq. wdot, with the 2/dx factor that the mapping
eq. x-xi implies; the printed dx/2 is read as its inverse):

  M_l dw_l/dt = (2/h) [ sum_q w_q sum_a f_a(u_q) . d_a phi_l(xi_q)
                        - sum_faces sum_r w_r F*(u_L, u_R) . phi_l(xi_r) n ]
                + sources,

with (d+1)-point Gauss-Legendre rules for the volume and the faces.
Powell (Sec. 4.1.3, eq. powell-src-face with q-dagger = q(<u>_K),
eq. powellq-average): each cell adds
  -(2/h) sum_faces sum_r w_r (q(<u>_K) . phi_l)(B^n_F - B^n_K)
with the outward normal; optionally (eq. powellq-interp) q-dagger varies over
the face points, q integrated along the straight path in primitive variables
from the cell's own trace to the HLLD interface state.  GLM (Sec. 4.1.5): psi flux and damping source
-kappa psi, kappa = c_h^2 / c_p^2.

Time step (Sec. 3.6, eq. cfl; Sec. 4.1.4, eq. powell_dt; Sec. 4.1.5 for c_h,
c_p), SSP-RK3 in Shu-Osher form (Sec. 3.6; Gottlieb et al. 2005).

Readings of the paper taken here (each also listed with the design notes):
 * c^K is the max over the cell's volume and face points of sum_a(|v_a|+c),
   c = sqrt(gamma p/rho + B^2/rho);
 * adaptive c_h = (C'/C) max_K sum_a(|v_a|+c) / D with C' = min(2C, 0.9),
   from u^n before the first stage; kappa = min(c_h/c_r, 1/(3 dt));
 * fixed c_h (AMR): dt also <= C' h_min / ((2d+1) D c_h);
 * Powell dt cap uses |div B|_K of eq. divb-cell (face-jump part for the LDF
   basis) and E, v.B at the cell average.

Mesh: a list of cells with sizes h_K and a list of faces (axis, left cell,
right cell, sub-face position on each side).  A full face has sub-face -1; a
quarter of a coarse face (2:1 hanging face) has sub-face j in 0..3 and the
coarse side evaluates its trace at xi_t = (xi_t^GL +- 1)/2 with weights
w_r / 4 (w_r / 2 in 2-D).  Uniform periodic grids use full faces only.
"""
import numpy as np

from . import basis as B
from . import physics as ph
from .quadrature import gauss_legendre, tensor_rule

GLM, POWELL = 0, 1


def ssp_rk(stages):
    """Shu-Osher coefficients (alpha, beta) of the SSP Runge-Kutta schemes of
    selectable order 1-4 (Sec. 3.6, citing the Gottlieb 2005 survey):
    u_i = sum_{j<i} alpha[i-1][j] u_j + beta[i-1][j] dt L(u_j), u_0 = u^n,
    u^{n+1} = u_s.  stages 1, 2, 3: the s-stage order-s schemes (forward Euler,
    SSP-RK2, Shu-Osher SSP-RK3); 5: the five-stage fourth-order scheme of
    Spiteri & Ruuth as listed in that survey (15 digits)."""
    if stages == 1:
        return [[1.0]], [[1.0]]
    if stages == 2:
        return [[1.0], [0.5, 0.5]], [[1.0], [0.0, 0.5]]
    if stages == 3:
        return ([[1.0], [0.75, 0.25], [1.0 / 3.0, 0.0, 2.0 / 3.0]],
                [[1.0], [0.0, 0.25], [0.0, 0.0, 2.0 / 3.0]])
    if stages == 5:
        alpha = [[1.0],
                 [0.444370493651235, 0.555629506348765],
                 [0.620101851488403, 0.0, 0.379898148511597],
                 [0.178079954393132, 0.0, 0.0, 0.821920045606868],
                 [0.0, 0.0, 0.517231671970585, 0.096059710526147, 0.386708617503269]]
        beta = [[0.391752226571890],
                [0.0, 0.368410593050371],
                [0.0, 0.0, 0.251891774271694],
                [0.0, 0.0, 0.0, 0.544974750228521],
                [0.0, 0.0, 0.0, 0.063692468666290, 0.226007483236906]]
        return alpha, beta
    raise ValueError("stages must be 1, 2, 3 or 5")


class Mesh:
    """Cells (centres, sizes) and faces of a periodic box."""

    def __init__(self, D, h, centers, faces):
        self.D = D
        self.h = np.asarray(h, dtype=np.float64)          # [C]
        self.centers = np.asarray(centers, dtype=np.float64)  # [C, D]
        self.faces = faces  # list of dicts: axis, L, R, subL, subR (int arrays)
        self.ncells = self.h.shape[0]

    @staticmethod
    def uniform(D, n, box=1.0):
        """n^D periodic cells on [0, box]^D; cell index i + n (j + n k)."""
        C = n ** D
        idx = np.arange(C)
        ijk = [(idx // n ** a) % n for a in range(D)]
        h = box / n
        centers = np.stack([(ijk[a] + 0.5) * h for a in range(D)], axis=1)
        faces = []
        for a in range(D):
            nb = idx + (((ijk[a] + 1) % n) - ijk[a]) * n ** a
            faces.append(dict(axis=a, L=idx.copy(), R=nb, subL=np.full(C, -1), subR=np.full(C, -1)))
        m = Mesh(D, np.full(C, h), centers, faces)
        m.n = n
        m.box = box
        return m

    def neighbor(self, a, s):
        """Uniform grid: index of the face neighbour along axis a, side s = +-1."""
        for f in self.faces:
            if f["axis"] == a:
                out = np.empty(self.ncells, dtype=np.int64)
                if s > 0:
                    out[f["L"]] = f["R"]
                else:
                    out[f["R"]] = f["L"]
                return out
        raise KeyError(a)


class DG:
    """Oracle DG scheme on a Mesh.  State layout: w[cell, mode] where the mode
    index is v*n + l for the Legendre-expanded variables, followed (Powell) by
    the N_div LDF weights of the magnetic field."""

    def __init__(self, mesh, d, divb=GLM, gamma=5.0 / 3.0, cfl=0.3, cfl_glm=None, glm_cr=0.18,
                 glm_ch_fixed=0.0, powell_eta=0.2, powell_q="mean"):
        """powell_q: the state q-dagger of the Powell face term, "mean"
        (q of the cell average, eq. powellq-average) or "interp" (eq.
        powellq-interp, with the HLLD interface state)."""
        D = mesh.D
        self.mesh, self.D, self.d = mesh, D, d
        self.divb, self.gamma, self.cfl = divb, gamma, cfl
        self.cfl_glm = cfl_glm if cfl_glm is not None else min(2.0 * cfl, 0.9)
        self.glm_cr, self.glm_ch_fixed, self.powell_eta = glm_cr, glm_ch_fixed, powell_eta
        if powell_q not in ("mean", "interp"):
            raise ValueError(powell_q)
        self.powell_q = powell_q
        self.n = B.n_modes(D, d)
        P = d + 1
        self.P = P
        # variables expanded on the Legendre basis
        if divb == GLM:
            self.nvar = 9
            self.leg_vars = list(range(9))
            self.nldf = 0
        else:
            self.nvar = 8
            self.leg_vars = [0, 1, 2, 3, 4] + [ph.B1 + c for c in range(D, 3)]
            self.nldf = B.n_div(D, d)
        self.nmodes = len(self.leg_vars) * self.n + self.nldf
        # volume rule and tables
        self.xq, self.wq = tensor_rule(P, D)
        self.V = B.legendre_values(D, d, self.xq)          # [Q, n]
        self.G = B.legendre_grads(D, d, self.xq)           # [D, Q, n]
        self.Mleg = B.legendre_mass(D, d)
        # face rule: tangential points of a full face
        xg, wg = gauss_legendre(P)
        if D == 2:
            self.xt = xg[:, None]
            self.wf = wg.copy()
        else:
            self.xt, self.wf = tensor_rule(P, 2)
        self.Fp = self.wf.shape[0]
        if self.nldf:
            self.Phi = B.ldf_values(D, d, self.xq)          # [D, Q, Nd]
            self.dPhi = B.ldf_grads(D, d, self.xq)          # [D(a), D(c), Q, Nd]
            self.Mldf = B.ldf_mass(D, d)
            self.ldf_mean = np.einsum("q,cql->cl", self.wq, self.Phi) / 2.0 ** D  # [D, Nd]
        self.M = np.concatenate([np.tile(self.Mleg, len(self.leg_vars))] +
                                ([self.Mldf] if self.nldf else []))
        self._face_tab = {}

    # ------------------------------------------------------------------
    # reference points on faces

    def face_points(self, a, side, sub):
        """Reference coordinates [Fp, D] of the face points of the face of a
        cell with outward normal side*e_a; sub = -1 full face, else quarter."""
        key = (a, side, sub)
        if key not in self._face_tab:
            D = self.D
            xi = np.empty((self.Fp, D))
            tang = [b for b in range(D) if b != a]
            xi[:, a] = float(side)
            for j, b in enumerate(tang):
                t = self.xt[:, j].copy()
                if sub >= 0:
                    off = ((sub >> j) & 1) * 2 - 1  # -1 or +1
                    t = 0.5 * (t + off)
                xi[:, b] = t
            self._face_tab[key] = xi
        return self._face_tab[key]

    def sub_weight(self, sub):
        if sub < 0:
            return 1.0
        return 0.5 ** (self.D - 1)

    # ------------------------------------------------------------------
    # modal -> nodal

    def _basis_at(self, xi):
        Vl = B.legendre_values(self.D, self.d, xi)
        Phi = B.ldf_values(self.D, self.d, xi) if self.nldf else None
        return Vl, Phi

    def nodal(self, w, xi=None, tabs=None):
        """u[var, cell, point] at reference points xi (default: volume points)."""
        if tabs is None:
            tabs = (self.V, self.Phi if self.nldf else None) if xi is None else self._basis_at(xi)
        Vl, Phi = tabs
        C = w.shape[0]
        U = np.zeros((self.nvar, C, Vl.shape[0]))
        n = self.n
        for j, v in enumerate(self.leg_vars):
            U[v] = w[:, j * n:(j + 1) * n] @ Vl.T
        if self.nldf:
            wb = w[:, len(self.leg_vars) * n:]
            for c in range(self.D):
                U[ph.B1 + c] = wb @ Phi[c].T
        return U

    def cell_means(self, w):
        """Cell-average conserved state [var, cell]."""
        C = w.shape[0]
        Ub = np.zeros((self.nvar, C))
        for j, v in enumerate(self.leg_vars):
            Ub[v] = w[:, j * self.n]
        if self.nldf:
            wb = w[:, len(self.leg_vars) * self.n:]
            for c in range(self.D):
                Ub[ph.B1 + c] = wb @ self.ldf_mean[c]
        return Ub

    def project_test(self, vals, tabs, weights):
        """sum_r weights_r vals[var, cell, r] . phi_m(r) -> [cell, mode]."""
        Vl, Phi = tabs
        C = vals.shape[1]
        out = np.zeros((C, self.nmodes))
        n = self.n
        for j, v in enumerate(self.leg_vars):
            out[:, j * n:(j + 1) * n] = (vals[v] * weights) @ Vl
        if self.nldf:
            o = len(self.leg_vars) * n
            for c in range(self.D):
                out[:, o:] += (vals[ph.B1 + c] * weights) @ Phi[c]
        return out

    # ------------------------------------------------------------------
    # right-hand side

    def rhs(self, w, ch=0.0, kappa=0.0):
        """dw/dt = R(w) / M  for the whole mesh (eq. wdot)."""
        mesh, D, g = self.mesh, self.D, self.gamma
        glm = self.divb == GLM
        C = w.shape[0]
        h = mesh.h
        R = np.zeros((C, self.nmodes))
        # volume integral
        U = self.nodal(w)
        n = self.n
        for a in range(D):
            Fa = ph.flux(U, a, g, glm, ch)
            for j, v in enumerate(self.leg_vars):
                R[:, j * n:(j + 1) * n] += (Fa[v] * self.wq) @ self.G[a]
            if self.nldf:
                o = len(self.leg_vars) * n
                for c in range(D):
                    R[:, o:] += (Fa[ph.B1 + c] * self.wq) @ self.dPhi[a, c]
        R *= (2.0 / h)[:, None]
        # faces
        Ub = self.cell_means(w) if self.divb == POWELL else None
        for f in mesh.faces:
            a = f["axis"]
            for subL in np.unique(f["subL"]):
                for subR in np.unique(f["subR"]):
                    sel = (f["subL"] == subL) & (f["subR"] == subR)
                    if not sel.any():
                        continue
                    L, Rc = f["L"][sel], f["R"][sel]
                    tL = self._basis_at(self.face_points(a, +1, subL))
                    tR = self._basis_at(self.face_points(a, -1, subR))
                    UL = self.nodal(w[L], tabs=tL)
                    UR = self.nodal(w[Rc], tabs=tR)
                    interp = self.divb == POWELL and self.powell_q == "interp"
                    if interp:
                        Fs, bnF, vF, BF = ph.numerical_flux(UL, UR, a, g, glm, ch, state=True)
                    else:
                        Fs, bnF = ph.numerical_flux(UL, UR, a, g, glm, ch)
                    wL = self.wf * self.sub_weight(subL)
                    wR = self.wf * self.sub_weight(subR)
                    cL = self.project_test(Fs, tL, wL) * (2.0 / h[L])[:, None]
                    cR = self.project_test(Fs, tR, wR) * (2.0 / h[Rc])[:, None]
                    np.subtract.at(R, L, cL)
                    np.add.at(R, Rc, cR)
                    if self.divb == POWELL:
                        jL = bnF - UL[ph.B1 + a]     # B^n_F - B^n_L (outward +e_a)
                        jR = UR[ph.B1 + a] - bnF     # (-B^n_F) - (-B^n_R)
                        if interp:
                            qL = ph.powell_q_interp(UL, vF, BF) * jL[None]
                            qR = ph.powell_q_interp(UR, vF, BF) * jR[None]
                        else:
                            qL = ph.powell_q(Ub[:, L])[:, :, None] * jL[None]
                            qR = ph.powell_q(Ub[:, Rc])[:, :, None] * jR[None]
                        pL = self.project_test(qL, tL, wL) * (2.0 / h[L])[:, None]
                        pR = self.project_test(qR, tR, wR) * (2.0 / h[Rc])[:, None]
                        np.subtract.at(R, L, pL)
                        np.subtract.at(R, Rc, pR)
        if glm:
            j = self.leg_vars.index(ph.PSI)
            R[:, j * n:(j + 1) * n] -= kappa * self.Mleg[None, :] * w[:, j * n:(j + 1) * n]
        return R / self.M[None, :]

    # ------------------------------------------------------------------
    # time step

    def all_point_states(self, w):
        """States at every volume and face point of every cell: list of [var, cell, p]."""
        out = [self.nodal(w)]
        for a in range(self.D):
            for s in (-1, 1):
                out.append(self.nodal(w, tabs=self._basis_at(self.face_points(a, s, -1))))
        return out

    def max_signal(self, w):
        """Per cell: max over volume and face points of sum_a (|v_a| + c)."""
        s = None
        for U in self.all_point_states(w):
            m = ph.signal_speed_sum(U, self.gamma, self.D).max(axis=1)
            s = m if s is None else np.maximum(s, m)
        return s

    def divb_face_jump(self, w):
        """Face-jump part of |div B|_K (eq. divb-cell): (1/V_K) int |B^n_F - B^n| dS."""
        mesh = self.mesh
        acc = np.zeros(mesh.ncells)
        for f in mesh.faces:
            a = f["axis"]
            for subL in np.unique(f["subL"]):
                for subR in np.unique(f["subR"]):
                    sel = (f["subL"] == subL) & (f["subR"] == subR)
                    if not sel.any():
                        continue
                    L, Rc = f["L"][sel], f["R"][sel]
                    UL = self.nodal(w[L], tabs=self._basis_at(self.face_points(a, +1, subL)))
                    UR = self.nodal(w[Rc], tabs=self._basis_at(self.face_points(a, -1, subR)))
                    bnF = ph.face_normal_field(UL[ph.B1 + a], UL[ph.RHO], UR[ph.B1 + a], UR[ph.RHO])
                    # reference face area element: dS = (h/2)^(D-1) dS_xi
                    jl = (np.abs(bnF - UL[ph.B1 + a]) * self.wf * self.sub_weight(subL)).sum(axis=1)
                    jr = (np.abs(UR[ph.B1 + a] - bnF) * self.wf * self.sub_weight(subR)).sum(axis=1)
                    hL, hR = mesh.h[L], mesh.h[Rc]
                    np.add.at(acc, L, jl * (hL / 2) ** (self.D - 1) / hL ** self.D)
                    np.add.at(acc, Rc, jr * (hR / 2) ** (self.D - 1) / hR ** self.D)
        return acc

    def timestep(self, w):
        """(dt, c_h, kappa) from the state at the start of a step."""
        D, d = self.D, self.d
        s = self.max_signal(w)
        h = self.mesh.h
        dt = self.cfl / (2 * d + 1) * np.min(h / s)
        ch = kappa = 0.0
        if self.divb == GLM:
            if self.glm_ch_fixed > 0.0:
                ch = self.glm_ch_fixed
                dt = min(dt, self.cfl_glm * h.min() / ((2 * d + 1) * D * ch))
            else:
                ch = (self.cfl_glm / self.cfl) * s.max() / D
            kappa = min(ch / self.glm_cr, 1.0 / (3.0 * dt))
        else:
            div = self.divb_face_jump(w)
            Ub = self.cell_means(w)
            vB = (Ub[ph.M1] * Ub[ph.B1] + Ub[ph.M2] * Ub[ph.B2] + Ub[ph.M3] * Ub[ph.B3]) / Ub[ph.RHO]
            prod = div * np.abs(vB)
            ok = prod > 0.0
            if ok.any():
                dt = min(dt, float(np.min(self.powell_eta * Ub[ph.EN][ok] / prod[ok])))
        return dt, ch, kappa

    # ------------------------------------------------------------------
    # SSP-RK3

    def step(self, w, limiter=None, rk=3):
        """One step of the SSP Runge-Kutta scheme with `rk` stages (ssp_rk; the
        default is SSP-RK3), in Shu-Osher form.  limiter(w, ch) -> w is applied
        after every stage with the step's c_h.  Returns (w_new, dt, ch, kappa)."""
        dt, ch, kappa = self.timestep(w)
        lim = (lambda x: limiter(x, ch)) if limiter is not None else (lambda x: x)
        alpha, beta = ssp_rk(rk)
        us, dls = [w], []
        for i in range(len(alpha)):
            dls.append(dt * self.rhs(us[-1], ch, kappa))
            u = sum(alpha[i][j] * us[j] + beta[i][j] * dls[j] for j in range(i + 1))
            us.append(lim(u))
        return us[-1], dt, ch, kappa

    # ------------------------------------------------------------------
    # initial-condition projection (d+3 points per dimension)

    def project(self, field, nq=None):
        """L2 projection of a pointwise conserved field onto the DG space:
        w_l = M_l^-1 sum_q w_q u(x_q) . phi_l(xi_q) with (d+3)^D GL points.
        field(x[P, D]) -> U[var, P]."""
        nq = nq if nq is not None else self.d + 3
        xq, wq = tensor_rule(nq, self.D)
        tabs = self._basis_at(xq)
        mesh = self.mesh
        x = mesh.centers[:, None, :] + 0.5 * mesh.h[:, None, None] * xq[None, :, :]
        U = field(x.reshape(-1, self.D)).reshape(self.nvar, mesh.ncells, xq.shape[0])
        return self.project_test(U, tabs, wq) / self.M[None, :]

    # ------------------------------------------------------------------
    # layout helpers for the C ABI ([mode][cell])

    def to_abi(self, w, ld=None):
        C = w.shape[0]
        ld = ld if ld is not None else C
        out = np.zeros((self.nmodes, ld))
        out[:, :C] = w.T
        return out

    def from_abi(self, a):
        return np.ascontiguousarray(a[:, :self.mesh.ncells].T)


def conserved_field(prim_fun, gamma, nvar, **kw):
    """Wrap a pointwise primitive field (dict rho, v, p, B, psi) as a conserved
    field x[P, D] -> U[nvar, P] for DG.project."""
    def f(x):
        pr = prim_fun(x, **kw)
        psi = pr.get("psi", 0.0) if nvar == 9 else None
        if psi is not None:
            psi = np.broadcast_to(np.asarray(psi, dtype=np.float64), np.shape(pr["rho"]))
        return ph.prim_to_cons(pr["rho"], pr["v"], pr["p"], pr["B"], gamma, psi)
    return f
