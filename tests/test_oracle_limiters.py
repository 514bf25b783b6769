"""Pins of the oracle's limiters and eigensystem (no GPU): the statements of
Sec. 4.2-4.3 (means kept, linear data untouched, positivity at every point,
tau = 1 leaves the cell bitwise unchanged, LDF fix divergence-free and
non-increasing), and L A R = diag(lambda) against a finite-difference flux
Jacobian."""
import numpy as np
import pytest

import workloads as wl
from oracle import dg, eigen, limiters
from oracle import physics as ph
from oracle.quadrature import tensor_rule

G = 5.0 / 3.0


def test_minmod_and_tvb_sigma():
    a = np.array([1.0, -1.0, 1.0, 0.5, 3.0])
    b = np.array([2.0, -0.5, -1.0, 0.2, 4.0])
    c = np.array([3.0, -2.0, 2.0, 0.9, 5.0])
    assert np.array_equal(limiters.minmod(a, b, c), [1.0, -0.5, 0.0, 0.2, 3.0])
    # linear data never changes: minmod(a, 2a, 2a) = a
    x = np.linspace(-2, 2, 9)
    assert np.array_equal(limiters.tvb_sigma(x, x, x, 0.0, 0.1, 2.0), x)
    # below the threshold |a| <= M~ h the slope is kept even at an extremum
    assert limiters.tvb_sigma(np.array([0.4]), np.array([1.0]), np.array([-1.0]), 5.0, 0.1, 2.0)[0] == 0.4
    assert limiters.tvb_sigma(np.array([0.6]), np.array([1.0]), np.array([-1.0]), 5.0, 0.1, 2.0)[0] == 0.0


def _fd_jacobian7(u, a, bn):
    perm = eigen.frame_permutation(a)[:8]
    sel = [0, 1, 2, 3, 4, 6, 7]

    def F7(x7):
        uf = np.zeros(8)
        uf[sel] = x7
        uf[5] = bn
        ug = np.zeros(8)
        ug[perm] = uf
        return ph.flux(ug[:, None], a, G)[:, 0][perm][sel]
    uf = u[perm][sel]
    J = np.zeros((7, 7))
    for k in range(7):
        e = np.zeros(7)
        hh = 1e-6 * max(1.0, abs(uf[k]))
        e[k] = hh
        J[:, k] = (F7(uf + e) - F7(uf - e)) / (2 * hh)
    return J


@pytest.mark.parametrize("kind", ["generic", "bt_zero", "bn_zero", "triple"])
def test_eigensystem_diagonalises_flux_jacobian(kind):
    rng = np.random.default_rng({"generic": 1, "bt_zero": 2, "bn_zero": 3, "triple": 4}[kind])
    for _ in range(4):
        rho, v, p, B = rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(0.1, 2), rng.uniform(-1, 1, 3)
        for a in range(3):
            BB = B.copy()
            n, t1, t2 = ph.face_frame(a)
            if kind == "bt_zero":
                BB[t1] = BB[t2] = 0.0
            if kind == "bn_zero":
                BB[n] = 0.0
            if kind == "triple":
                BB[t1] = BB[t2] = 0.0
                BB[n] = np.sqrt(G * p)  # c_A = a
            u = ph.prim_to_cons(np.array(rho), v, np.array(p), BB, G, np.array(0.2))
            L, R = eigen.char_matrices(u, a, G, 1.7)
            assert np.abs(L @ R - np.eye(9)).max() < 1e-12
            assert np.linalg.cond(R) < 1e4
            perm = eigen.frame_permutation(a)
            rows = [perm[i] for i in eigen.IDX7]
            J = _fd_jacobian7(u[:8], a, u[perm[5]])
            Dm = L[eigen.IDX7][:, rows] @ J @ R[rows][:, eigen.IDX7]
            off = Dm - np.diag(np.diag(Dm))
            assert np.abs(off).max() < 1e-7 * max(1.0, np.abs(Dm).max())
            # eigenvalues sorted u-cf <= u-ca <= u-cs <= u <= ...
            lam = np.diag(Dm)
            assert np.all(np.diff(lam) > -1e-7)
            # GLM pair (B_n, psi): L_g [[0, 1], [c_h^2, 0]] R_g = diag(c_h, -c_h)
            gi = [perm[5], perm[8]]
            A2 = np.array([[0.0, 1.0], [1.7 ** 2, 0.0]])
            cols = [i for i in range(9) if np.abs(R[gi, i]).max() > 0 and i not in eigen.IDX7]
            Dg = L[np.ix_(cols, gi)] @ A2 @ R[np.ix_(gi, cols)]
            assert np.allclose(Dg, np.diag([1.7, -1.7]), atol=1e-14)


@pytest.mark.parametrize("a2_over_ca2", [0.5, 2.0])
def test_eigenvectors_are_continuous_at_rounding_level_near_degenerate_states(a2_over_ca2):
    """At B_t = 0 (and at B_n = 0) the characteristic matrices move by no
    more than the state does: a relative change of 1e-15 in p, rho or the
    field must not shift them by the square root of rounding (~1e-8), which a
    fast/slow normalisation formed by cancellation does."""
    rho, p = 1.3, 0.7
    bn = np.sqrt(G * p / a2_over_ca2 * rho)      # c_a^2 = a^2 / ratio
    v = np.array([0.1, -0.2, 0.3])
    for a in range(3):
        n, t1, t2 = ph.face_frame(a)
        for kind in ("bt_zero", "bn_zero"):
            B0 = np.zeros(3)
            B0[n if kind == "bt_zero" else t1] = bn
            base = ph.prim_to_cons(np.array(rho), v, np.array(p), B0, G, np.array(0.0))
            L0, R0 = eigen.char_matrices(base, a, G, 1.0)
            for k in range(6):
                r, pp, B1 = rho, p, B0.copy()
                pert = 1e-15 * (k + 1)
                if k % 3 == 0:
                    pp = p * (1 + pert)
                elif k % 3 == 1:
                    r = rho * (1 + pert)
                else:
                    B1[t1 if kind == "bt_zero" else n] += pert
                u1 = ph.prim_to_cons(np.array(r), v, np.array(pp), B1, G, np.array(0.0))
                L1, R1 = eigen.char_matrices(u1, a, G, 1.0)
                assert np.abs(R1 - R0).max() < 1e-11, (a, kind, k, np.abs(R1 - R0).max())
                assert np.abs(L1 - L0).max() < 1e-11, (a, kind, k, np.abs(L1 - L0).max())


def test_characteristic_matrices_are_used_only_where_they_are_well_conditioned():
    """char_usable accepts a mean state exactly when gamma p >= 1e-8 (gamma p
    + |B|^2); on the accepted side the condition number of R stays below
    ~1e9 (it grows like |B|^2 / (gamma p)), on the rejected side it exceeds
    ~1e8 and L R = I fails at low pressures; NaN and non-positive states are
    rejected."""
    b = 100.0 / np.sqrt(3.0) / np.sqrt(4.0 * np.pi)
    B = np.array([b, 1.01 * b, 0.99 * b])
    g = 1.4
    for p in (1e-1, 1e-3, 1e-5, 2e-6, 1e-7, 1e-9, 1e-12):
        u = ph.prim_to_cons(np.array(1.0), np.array([0.3, -0.2, 0.1]), np.array(p), B, g, np.array(0.0))
        ok = limiters.char_usable(u, g)
        assert ok == (g * p >= 1e-8 * (g * p + (B ** 2).sum()))
        L, R = eigen.char_matrices(u, 0, g, 50.0)
        cond = np.linalg.cond(R)
        assert (cond < 1e9) if ok else (cond > 1e8)
    bad = ph.prim_to_cons(np.array(1.0), np.zeros(3), np.array(0.1), B, g, np.array(0.0))
    for k, val in ((0, -1.0), (4, 0.0), (4, np.nan)):
        v = bad.copy()
        v[k] = val
        assert not limiters.char_usable(v, g)


def test_floor_level_cells_are_limited_componentwise():
    """A strong-field state whose pressure sits at the floor in some cells:
    the characteristic limiter returns finite weights, and in those cells the
    limited slopes equal the componentwise limiter's."""
    s = dg.DG(dg.Mesh.uniform(2, 12), 2, gamma=1.4)
    b = 100.0 / np.sqrt(3.0) / np.sqrt(4.0 * np.pi)

    def prim(x):
        r = np.hypot(x[:, 0] - 0.5, x[:, 1] - 0.5)
        one = np.ones(x.shape[0])
        p = np.where(r < 0.15, 1000.0, np.where(r < 0.4, 1e-12, 0.1)) * one
        return dict(rho=1.0 + 0.5 * (r < 0.15), v=[0.3 * one, 0 * one, 0 * one], p=p, B=[b * one, b * one, b * one],
                    psi=0 * one)
    w = s.project(dg.conserved_field(prim, 1.4, 9))
    means = s.cell_means(w)
    low = np.array([not limiters.char_usable(means[:, k], 1.4) for k in range(w.shape[0])])
    assert low.any() and not low.all()
    wc, tc = limiters.slope_limit(s, w, characteristic=True, ch=30.0)
    wp, tp = limiters.slope_limit(s, w, characteristic=False, ch=30.0)
    assert np.all(np.isfinite(wc))
    assert np.array_equal(wc[low], wp[low]) and np.array_equal(tc[low], tp[low])


def _at_floor_state(divb=dg.GLM, seed=5):
    """Strong-field state whose cells have their mean pressure set exactly at
    the floor (the energy mode written from the means) while their slopes
    stay, so that points lie on both sides of the mean and of the floor."""
    s = dg.DG(dg.Mesh.uniform(2, 8), 2, divb=divb, gamma=1.4)
    rng = np.random.default_rng(seed)
    b = 16.0

    def prim(x):
        one = np.ones(x.shape[0])
        return dict(rho=1.0 + 0.3 * np.sin(2 * np.pi * x[:, 0]), v=[0.2 * np.cos(2 * np.pi * x[:, 1]), 0 * one, 0 * one],
                    p=0.1 * one, B=[b * one, b * one, b * one], psi=0 * one)
    w = s.project(dg.conserved_field(prim, 1.4, s.nvar))
    C, n = w.shape[0], s.n
    eidx = s.leg_vars.index(ph.EN) * n
    cells = rng.permutation(C)[:C // 2]
    w[cells, eidx + 1:eidx + n] += 1e-12 * rng.normal(size=(cells.size, n - 1))
    Ub = s.cell_means(w)
    ke = 0.5 * (Ub[1] ** 2 + Ub[2] ** 2 + Ub[3] ** 2) / Ub[0]
    me = 0.5 * (Ub[5] ** 2 + Ub[6] ** 2 + Ub[7] ** 2)
    w[cells, eidx] = 1e-12 / 0.4 + ke[cells] + me[cells]
    return s, w, cells


def test_point_tau_rule():
    """The per-point factor: the closed form (mean - floor)/(mean - q) for a
    point below both; 1 for a point at or above the mean (including a point
    equal to the mean, where the ratio would be 0/0 or +-inf) and for
    unmasked points; a mean below the floor gives a negative factor, which
    the cell's tau clips to 0."""
    mean = np.array([1.0, 1.0, 1e-12, 1e-12, 0.9e-12, 0.5])
    q = np.array([-0.5, 2.0, 1e-12, 0.5e-12, 0.5e-12, -1.0])
    mask = np.array([True, True, True, True, True, False])
    t = limiters.point_tau(mean, q, 1e-12, mask)
    assert np.isclose(t[0], (1.0 - 1e-12) / 1.5, rtol=1e-15)
    assert t[1] == 1.0 and t[2] == 1.0 and t[5] == 1.0
    assert t[3] == 0.0
    assert t[4] < 0.0 and np.isfinite(t).all()


@pytest.mark.parametrize("divb", [dg.GLM, dg.POWELL])
def test_positivity_with_means_at_the_floor_is_finite_and_convex(divb):
    """Eq. tau_press with the mean pressure at the floor (up to the rounding
    of E - |m|^2/2rho - |B|^2/2 ~ 5e-14): every cell's new weights are its
    mean plus tau times its deviation with tau in [0, 1] (no sign flip, no
    infinity from a point equal to the mean), and all are finite."""
    s, w, cells = _at_floor_state(divb)
    w2, st = limiters.positivity(s, w)
    assert np.all(np.isfinite(w2))
    assert st["n_pos_scaled"] > 0
    n = s.n
    keep = np.zeros(w.shape[1], dtype=bool)
    keep[[j * n for j in range(len(s.leg_vars))]] = True
    if s.nldf:
        keep[len(s.leg_vars) * n:len(s.leg_vars) * n + s.D] = True
    for k in range(w.shape[0]):
        dv, dv2 = w[k, ~keep], w2[k, ~keep]
        big = np.abs(dv) > 0
        if not big.any():
            continue
        r = dv2[big] / dv[big]
        assert np.all(r >= -1e-15) and np.all(r <= 1 + 1e-15), (k, r.min(), r.max())
        assert np.ptp(r) < 1e-12                           # one tau per cell


def _blast_state(n=6, d=2, seed=2000):
    s = dg.DG(dg.Mesh.uniform(3, n), d)
    w = s.project(dg.conserved_field(wl.Blast(seed), G, 9))
    return s, w


def test_slope_limiter_keeps_means_and_untriggered_cells():
    s, w = _blast_state()
    w2, tr = limiters.slope_limit(s, w, ch=2.0)
    assert tr.any() and not tr.all()
    mean_cols = [v * s.n for v in range(9)]
    assert np.array_equal(w2[:, mean_cols], w[:, mean_cols])
    assert np.array_equal(w2[~tr], w[~tr])
    hi = [v * s.n + l for v in range(9) for l in range(4, s.n)]
    assert np.all(w2[np.ix_(tr, hi)] == 0.0)


def test_slope_limiter_leaves_smooth_state_alone_with_large_threshold():
    s = dg.DG(dg.Mesh.uniform(2, 16), 2)
    w = s.project(dg.conserved_field(wl.Smooth(3, 2), G, 9))
    w2, tr = limiters.slope_limit(s, w, Mtilde=1e6, ch=2.0)
    assert not tr.any() and np.array_equal(w, w2)


def test_componentwise_mode_is_identity_eigensystem():
    s, w = _blast_state(n=5)
    w_c, tr_c = limiters.slope_limit(s, w, characteristic=False)
    # recompute by hand with L = R = I on one triggered cell
    c = int(np.argmax(tr_c))
    assert tr_c[c]
    n = s.n
    for a in range(3):
        up, dn = s.mesh.neighbor(a, 1)[c], s.mesh.neighbor(a, -1)[c]
        means = s.cell_means(w)
        for v in range(9):
            slope = w[c, v * n + 1 + a]
            sig = limiters.tvb_sigma(np.array([slope]), np.array([0.5 * (means[v, up] - means[v, c])]),
                                     np.array([0.5 * (means[v, c] - means[v, dn])]), 5.0, s.mesh.h[c], 2.0)[0]
            trig_dir = any(abs(limiters.tvb_sigma(
                np.array([w[c, vv * n + 1 + a]]), np.array([0.5 * (means[vv, up] - means[vv, c])]),
                np.array([0.5 * (means[vv, c] - means[vv, dn])]), 5.0, s.mesh.h[c], 2.0)[0] - w[c, vv * n + 1 + a])
                > 1e-8 for vv in range(9))
            want = sig if (trig_dir and abs(sig - slope) > 1e-8) else slope
            assert w_c[c, v * n + 1 + a] == pytest.approx(want, abs=1e-15)


def test_positivity_limiter_invariants():
    s, w = _blast_state(n=6, d=3)
    # make some points negative: sharpen the IC
    w = w.copy()
    hi = [4 * s.n + l for l in range(1, s.n)]
    w[:, hi] *= 3.0
    pts0 = np.concatenate(s.all_point_states(w), axis=2)
    assert (ph.pressure(pts0, G) < 0).any()
    w2, st = limiters.positivity(s, w)
    assert st["n_pos_scaled"] > 0 and st["n_floor"] == 0
    pts = np.concatenate(s.all_point_states(w2), axis=2)
    assert pts[ph.RHO].min() >= 1e-12 * (1 - 1e-9)
    assert ph.pressure(pts, G).min() >= -1e-13
    mean_cols = [v * s.n for v in range(9)]
    assert np.array_equal(w2[:, mean_cols], w[:, mean_cols])
    # tau = 1 cells are bitwise unchanged
    ok = (ph.pressure(pts0, G).min(axis=1) >= 1e-12) & (pts0[ph.RHO].min(axis=1) >= 1e-12)
    assert ok.any()
    assert np.array_equal(w2[ok], w[ok])


def test_positivity_floors_tally():
    s = dg.DG(dg.Mesh.uniform(2, 4), 1)
    w = s.project(dg.conserved_field(wl.Smooth(4, 2), G, 9))
    w[3, 0] = -0.5           # negative mean density (at rest, so only the density floor fires)
    w[3, [s.n, 2 * s.n, 3 * s.n]] = 0.0
    w[5, 4 * s.n] = 0.0      # zero total energy -> negative mean pressure
    w2, st = limiters.positivity(s, w)
    assert st["n_floor"] == 2
    assert st["injected_mass"] == pytest.approx((1e-12 + 0.5) * s.mesh.h[3] ** 2)
    assert st["injected_energy"] > 0
    Ub = s.cell_means(w2)
    assert Ub[0].min() >= 1e-12 and ph.pressure(Ub, G).min() >= 1e-12 * (1 - 1e-6)


def test_ldf_divergence_fix_invariants():
    rng = np.random.default_rng(9)
    for _ in range(50):
        S = rng.normal(size=(3, 3))
        S2 = limiters.ldf_divfree_fix(S)
        assert abs(np.trace(S2)) < 1e-14 * np.abs(S).max()
        assert np.all(np.abs(np.diag(S2)) <= np.abs(np.diag(S)) + 1e-15)
        off = ~np.eye(3, dtype=bool)
        assert np.array_equal(S2[off], S[off])
        # the untouched sign class keeps its slopes exactly
        d, d2 = np.diag(S), np.diag(S2)
        if np.trace(S) > 0:
            assert np.array_equal(d2[d <= 0], d[d <= 0])
        else:
            assert np.array_equal(d2[d >= 0], d[d >= 0])


def test_ldf_projection_of_divfree_linear_field_is_exact():
    s = dg.DG(dg.Mesh.uniform(3, 2), 2, divb=dg.POWELL)
    rng = np.random.default_rng(10)
    S = limiters.ldf_divfree_fix(rng.normal(size=(3, 3)))
    Bm = rng.normal(size=3)
    wl_ = limiters.ldf_project_linear(s, Bm, S)
    from oracle import basis as Bb
    degs = np.array(Bb.ldf_degrees(3, 2))
    assert np.abs(wl_[degs >= 2]).max() < 1e-14   # no higher-degree contamination
    xq, _ = tensor_rule(4, 3)
    Phi = Bb.ldf_values(3, 2, xq)
    Bq = np.einsum("cpl,l->cp", Phi, wl_)
    assert np.allclose(Bq, Bm[:, None] + S @ xq.T, atol=1e-13)


def _fd_jacobian_powell(u8, a):
    """A = dF/dU + q(U) e_{B_n}^T in the frame order (rho, m_n, m_t1, m_t2, E,
    B_n, B_t1, B_t2): the flux Jacobian along a with B_n a variable, plus the
    Powell source -q dB_n/dx written as a transport term (Sec. 4.1.3,
    eq. powell-src with q of eq. powell-q)."""
    perm = eigen.frame_permutation(a)[:8]

    def F8(uf):
        ug = np.zeros(8)
        ug[perm] = uf
        return ph.flux(ug[:, None], a, G)[:, 0][perm]
    uf = u8[perm]
    J = np.zeros((8, 8))
    for k in range(8):
        e = np.zeros(8)
        hh = 1e-6 * max(1.0, abs(uf[k]))
        e[k] = hh
        J[:, k] = (F8(uf + e) - F8(uf - e)) / (2 * hh)
    q = ph.powell_q(u8[:, None])[:, 0][perm]
    J[:, 5] += q
    return J


@pytest.mark.parametrize("kind", ["generic", "bt_zero", "bn_zero", "triple"])
def test_powell_eight_wave_system_diagonalises_the_powell_jacobian(kind):
    """Powell scheme (f1 of the scope): L A R = diag(lambda) with A the
    Jacobian of the Powell system and the eigenvalues u - c_f <= u - c_a <=
    u - c_s <= u <= u + c_s <= u + c_a <= u + c_f plus the divergence wave u."""
    rng = np.random.default_rng({"generic": 11, "bt_zero": 12, "bn_zero": 13, "triple": 14}[kind])
    for _ in range(4):
        rho, v, p, B = rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(0.1, 2), rng.uniform(-1, 1, 3)
        for a in range(3):
            BB = B.copy()
            n, t1, t2 = ph.face_frame(a)
            if kind == "bt_zero":
                BB[t1] = BB[t2] = 0.0
            if kind == "bn_zero":
                BB[n] = 0.0
            if kind == "triple":
                BB[t1] = BB[t2] = 0.0
                BB[n] = np.sqrt(G * p)
            u = ph.prim_to_cons(np.array(rho), v, np.array(p), BB, G)
            L, R = eigen.char_matrices(u, a, G, None, nvar=8)
            assert np.abs(L @ R - np.eye(8)).max() < 1e-12
            perm = eigen.frame_permutation(a)[:8]
            A = _fd_jacobian_powell(u, a)
            Dm = L[:, perm] @ A @ R[perm, :]
            off = Dm - np.diag(np.diag(Dm))
            assert np.abs(off).max() < 1e-7 * max(1.0, np.abs(Dm).max())
            lam = np.diag(Dm)
            un = v[n]
            # the divergence wave (B_n column of the frame) travels with the flow
            assert abs(lam[perm.index(ph.B1 + n)] - un) < 1e-7
            waves = np.sort(np.delete(lam, perm.index(ph.B1 + n)))
            assert abs(waves[3] - un) < 1e-7 and np.all(np.diff(waves) > -1e-7)


def _powell_blast(n=8, d=2, seed=2000):
    s = dg.DG(dg.Mesh.uniform(3, n), d, divb=dg.POWELL)
    w = s.project(dg.conserved_field(wl.Blast(seed), G, 8))
    return s, w


def test_powell_slope_limiter_invariants():
    """Powell + LDF limiting (Sec. 4.2.4): means unchanged; every troubled cell
    leaves a divergence-free linear magnetic field (its LDF weights are those
    of a linear field whose diagonal slopes sum to zero, up to rounding); cells
    not troubled are bitwise unchanged; linear data is left alone."""
    s, w = _powell_blast()
    w2, tr = limiters.slope_limit(s, w)
    assert tr.any() and not tr.all()
    assert np.array_equal(w2[~tr], w[~tr])
    m1, m2 = s.cell_means(w), s.cell_means(w2)
    assert np.allclose(m1, m2, rtol=0, atol=1e-13 * np.abs(m1).max())
    Pm, Pl = limiters.ldf_moments(s)
    nl = len(s.leg_vars) * s.n
    for k in np.nonzero(tr)[0]:
        S = np.einsum("cbl,l->cb", Pl, w2[k, nl:])
        assert abs(np.trace(S)) < 1e-12 * max(1.0, np.abs(S).max())
        # the limited field is linear: reprojecting its linear part gives it back
        back = limiters.ldf_project_linear(s, m2[ph.B1:ph.B1 + 3, k], S)
        assert np.allclose(back, w2[k, nl:], rtol=0, atol=1e-12 * max(1.0, np.abs(back).max()))
        # Legendre variables: no modes of degree >= 2 left
        for j in range(5):
            assert np.all(w2[k, j * s.n + 4:(j + 1) * s.n] == 0.0)
    # a linear state (every variable and the field linear, divergence-free) is not limited
    lin = np.array([1.2, 0.1, -0.2, 0.05, 3.0, 0.4, -0.3, 0.2])
    grad = np.array([[0.01, 0, 0], [0, 0.01, 0], [0, 0, 0.0], [0.0, 0, 0.01], [0.02, 0.01, 0],
                     [0.01, 0.02, 0], [0.03, -0.01, 0], [0, 0.01, 0.0]])   # field rows: trace zero

    def field(x):
        U = lin[:, None] + grad @ (x.T - 0.5)
        return {"rho": U[0], "v": [U[1] / U[0], U[2] / U[0], U[3] / U[0]], "p": np.full(x.shape[0], 1.0),
                "B": [U[5], U[6], U[7]]}
    s2 = dg.DG(dg.Mesh.uniform(3, 4, box=1.0), 1, divb=dg.POWELL)
    # a non-periodic linear field would jump at the box edge: keep it to the interior cells
    wl_ = s2.project(dg.conserved_field(field, G, 8))
    w3, tr3 = limiters.slope_limit(s2, wl_, Mtilde=0.0)
    ijk = [(np.arange(64) // 4 ** a) % 4 for a in range(3)]
    interior = np.all([(c >= 1) & (c <= 2) for c in ijk], axis=0)
    assert not tr3[interior].any()
