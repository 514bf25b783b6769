"""Seeded synthetic inputs for the DG MHD scheme.

This module only draws random numbers and evaluates analytic *primitive*
fields (rho, v, p, B, psi) at physical points.  It holds none of the scheme's
arithmetic: no quadrature, no basis, no projection, no equation of state.
Both the CPU oracle and the HIP library project these pointwise values onto
their own modal bases with their own code.

Every evaluator accepts numpy arrays or torch tensors (``xp`` is picked from
the input), so the same seeded field can be evaluated on the host for the
oracle and on the device for large runs.

Recipes (one per workload):
  smooth      rho = 1 + 0.1 S_rho, p = 1 + 0.1 S_p, v = 0.1 S_v,
              B = curl(0.1 S_A) with S a normalised random Fourier sum over
              integer wave vectors 1 <= |k| <= 4 (half space), amplitudes
              U(-1,1), phases U(0, 2 pi); draw order rho, p, vx, vy, vz, A.
  blast       rho = 1, p = 0.1, v = 0, B = (1, 0.5, 0.2)/sqrt(4 pi); 8 spheres
              (centres U[0,1)^3, radii U[0.05, 0.1], periodic distance) with
              p = 10 inside.
  peaks       rho = 1 + 9 sum_i exp(-|x - c_i|^2 / (2 * 0.03^2)) over 16 peaks
              (periodic distance), p = 1, v = (0.5, 0.25, 0.125),
              B = (1, 0.5, 0.2)/sqrt(4 pi): an exact entropy wave.
  alfven2d    circularly polarised Alfven wave of the paper's 2-D convergence
              test (box sqrt(5), eps = 0.1, p = 0.1), exact at any time.
  alfven3d    the 3-D variant along the cube diagonal (p = 100, eps = 0.02).

Shock problems of the paper's test section (deterministic, no random draws):
  orszag_tang [0,1]^2, rho = 25/(36 pi), p = 5/(12 pi), v = (-sin 2pi y,
              sin 2pi x, 0), B = B0 (-sin 2pi y, sin 4pi x, 0), B0 = 1/sqrt(4 pi).
  rotor       [0,1]^2, p = 1, B = (5/sqrt(4 pi), 0, 0); disk r < 0.1 with
              rho = 10 rotating at v = (0.5 - y, x - 0.5) v0/r0 (v0 = 2),
              linear taper f = (r1 - r)/(r1 - r0) to r1 = 0.115 (rho = 1 + 9f,
              v scaled by f), rho = 1 at rest outside.
  blast2d     [0,1]^2, rho = 1, p = 0.1, v = 0, B = B0 (cos 45, sin 45, 0),
              B0 = 1; p = 10 within r0 = 0.1 of the box centre.
  blast3d     [0,1]^3, rho = 1, p = 0.1, v = 0, B = (B0, B0, B0),
              B0 = 100/(sqrt 3 sqrt(4 pi)), gamma 1.4 (2p/|B|^2 = 2.5e-4;
              the plasma beta of 7.5e-4 the paper quotes is 2p/B0^2);
              p = 1000 within r0 = 0.1 of the centre, which sits half a cell
              off the box centre (at a cell centre).
  loop        [-1,1]^2 (mesh box 2, coordinates shifted by -1), rho = 1, p = 1,
              v = (2, 1, 0), B = curl (0, 0, A_z) with A_z = A0 max(0, r0 - r),
              A0 = 1e-3, r0 = 0.3: B = A0 (-y, x, 0)/r inside the loop.
"""
import math

import numpy as np

try:  # torch is optional here
    import torch
except Exception:  # pragma: no cover
    torch = None


def _xp(x):
    if torch is not None and isinstance(x, torch.Tensor):
        return torch
    return np


def _const(xp, like, val):
    if xp is np:
        return np.full(like.shape, float(val))
    return torch.full(like.shape, float(val), dtype=like.dtype, device=like.device)


def wave_vectors(D, kmax=4):
    """Integer k with 1 <= |k| <= kmax, first nonzero component > 0, lexicographic."""
    out = []
    rng = range(-kmax, kmax + 1)
    if D == 2:
        cand = [(a, b) for a in rng for b in rng]
    else:
        cand = [(a, b, c) for a in rng for b in rng for c in rng]
    for k in cand:
        n2 = sum(x * x for x in k)
        if n2 == 0 or n2 > kmax * kmax:
            continue
        first = next(x for x in k if x != 0)
        if first > 0:
            out.append(k)
    return np.array(out, dtype=np.float64)


class FourierField:
    """S(x) = sum_k a_k cos(2 pi k.x + phi_k) / sum_k |a_k| and its gradient."""

    def __init__(self, rng, D):
        self.k = wave_vectors(D)
        nk = self.k.shape[0]
        self.a = rng.uniform(-1.0, 1.0, nk)
        self.phi = rng.uniform(0.0, 2.0 * math.pi, nk)
        self.norm = np.abs(self.a).sum()

    def _arg(self, x):
        xp = _xp(x)
        k = self.k if xp is np else torch.as_tensor(self.k, dtype=x.dtype, device=x.device)
        phi = self.phi if xp is np else torch.as_tensor(self.phi, dtype=x.dtype, device=x.device)
        return 2.0 * math.pi * (x @ k.T) + phi, xp

    def value(self, x):
        arg, xp = self._arg(x)
        a = self.a if xp is np else torch.as_tensor(self.a, dtype=x.dtype, device=x.device)
        return (xp.cos(arg) @ a) / self.norm

    def grad(self, x):
        arg, xp = self._arg(x)
        a = self.a if xp is np else torch.as_tensor(self.a, dtype=x.dtype, device=x.device)
        k = self.k if xp is np else torch.as_tensor(self.k, dtype=x.dtype, device=x.device)
        s = -xp.sin(arg) * a  # [P, nk]
        return (2.0 * math.pi / self.norm) * (s @ k)  # [P, D]


class Smooth:
    """Smooth periodic MHD state on [0,1]^D (divergence-free B)."""

    def __init__(self, seed, D):
        rng = np.random.default_rng(seed)
        self.D = D
        self.rho = FourierField(rng, D)
        self.p = FourierField(rng, D)
        self.v = [FourierField(rng, D) for _ in range(3)]
        self.A = [FourierField(rng, D) for _ in range(1 if D == 2 else 3)]

    def __call__(self, x):
        """x[P, D] -> dict of primitive fields (each [P])."""
        xp = _xp(x)
        rho = 1.0 + 0.1 * self.rho.value(x)
        p = 1.0 + 0.1 * self.p.value(x)
        v = [0.1 * f.value(x) for f in self.v]
        if self.D == 2:
            gz = 0.1 * self.A[0].grad(x)
            Bv = [gz[:, 1], -gz[:, 0], _const(xp, rho, 0.0)]
        else:
            g = [0.1 * f.grad(x) for f in self.A]  # g[c][:, j] = d A_c / d x_j
            Bv = [g[2][:, 1] - g[1][:, 2], g[0][:, 2] - g[2][:, 0], g[1][:, 0] - g[0][:, 1]]
        return dict(rho=rho, v=v, p=p, B=Bv, psi=_const(xp, rho, 0.0))


def _periodic_d2(x, c):
    xp = _xp(x)
    d = x - c
    d = d - xp.round(d)
    return (d * d).sum(axis=-1) if xp is np else (d * d).sum(dim=-1)


class Blast:
    """Uniform magnetised medium with 8 over-pressured spheres in [0,1]^3."""

    B0 = (1.0 / math.sqrt(4 * math.pi), 0.5 / math.sqrt(4 * math.pi), 0.2 / math.sqrt(4 * math.pi))

    def __init__(self, seed, nsph=8, p_in=10.0, p_out=0.1):
        rng = np.random.default_rng(seed)
        self.c = rng.uniform(0.0, 1.0, (nsph, 3))
        self.r = rng.uniform(0.05, 0.1, nsph)
        self.p_in, self.p_out = p_in, p_out

    def __call__(self, x):
        xp = _xp(x)
        inside = None
        for c, r in zip(self.c, self.r):
            cc = c if xp is np else torch.as_tensor(c, dtype=x.dtype, device=x.device)
            m = _periodic_d2(x, cc) < r * r
            inside = m if inside is None else (inside | m)
        p = xp.where(inside, _const(xp, x[:, 0], self.p_in), _const(xp, x[:, 0], self.p_out))
        z = _const(xp, x[:, 0], 0.0)
        return dict(rho=_const(xp, x[:, 0], 1.0), v=[z, z, z], p=p,
                    B=[_const(xp, x[:, 0], b) for b in self.B0], psi=z)


class Peaks:
    """16 Gaussian density peaks advected by a uniform flow (exact entropy wave)."""

    B0 = Blast.B0
    V0 = (0.5, 0.25, 0.125)

    def __init__(self, seed, npk=16, width=0.03, contrast=10.0):
        rng = np.random.default_rng(seed)
        self.c = rng.uniform(0.0, 1.0, (npk, 3))
        self.width, self.amp = width, contrast - 1.0

    def __call__(self, x, t=0.0):
        xp = _xp(x)
        shift = np.array(self.V0) * t
        rho = _const(xp, x[:, 0], 1.0)
        for c in self.c:
            cc = (c + shift) % 1.0
            cc = cc if xp is np else torch.as_tensor(cc, dtype=x.dtype, device=x.device)
            rho = rho + self.amp * xp.exp(-_periodic_d2(x, cc) / (2.0 * self.width ** 2))
        return dict(rho=rho, v=[_const(xp, rho, u) for u in self.V0], p=_const(xp, rho, 1.0),
                    B=[_const(xp, rho, b) for b in self.B0], psi=_const(xp, rho, 0.0))

    def refine_flags(self, centers, radius):
        """Cells (by centre) within `radius` (periodic) of any peak at t = 0."""
        flag = np.zeros(centers.shape[0], dtype=bool)
        for c in self.c:
            flag |= _periodic_d2(centers, c) < radius * radius
        return flag


class Alfven2D:
    """Travelling circularly polarised Alfven wave in [0, sqrt 5]^2 (exact)."""

    def __init__(self, eps=0.1, p=0.1, m=2):
        self.alpha = math.atan(1.0 / m)
        self.L = 1.0 / math.sin(self.alpha)
        self.eps, self.p0 = eps, p

    def __call__(self, x, t=0.0):
        xp = _xp(x)
        ca, sa = math.cos(self.alpha), math.sin(self.alpha)
        # the wave moves with -v_A = -1 along the parallel direction
        xs, ys = x[:, 0] + t * ca, x[:, 1] + t * sa
        phase = 2.0 * math.pi * (xs * ca + ys * sa)
        e = self.eps
        bpar, bperp, bz = 1.0, e * xp.sin(phase), e * xp.cos(phase)
        vpar, vperp, vz = 0.0, e * xp.sin(phase), e * xp.cos(phase)
        one = _const(xp, phase, 1.0)
        Bx = bpar * ca * one - bperp * sa
        By = bpar * sa * one + bperp * ca
        vx = vpar * ca * one - vperp * sa
        vy = vpar * sa * one + vperp * ca
        return dict(rho=one, v=[vx, vy, vz], p=self.p0 * one, B=[Bx, By, bz], psi=0.0 * one)


class Alfven3D:
    """Circularly polarised Alfven wave along the diagonal of [0,1]^3 (exact)."""

    def __init__(self, eps=0.02, p=100.0):
        self.eps, self.p0 = eps, p
        e1 = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
        e2 = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)
        e3 = np.cross(e1, e2)
        self.E = np.stack([e1, e2, e3])  # rows: primed axes in unprimed coordinates
        self.lam = 1.0 / math.sqrt(3.0)

    def __call__(self, x, t=0.0):
        xp = _xp(x)
        e = self.eps
        E = self.E if xp is np else torch.as_tensor(self.E, dtype=x.dtype, device=x.device)
        xpar = x @ E[0]
        phase = 2.0 * math.pi / self.lam * (xpar - 2.0 * t)
        one = _const(xp, phase, 1.0)
        vprime = [one, e * xp.cos(phase), e * xp.sin(phase)]
        bprime = [one, -e * xp.cos(phase), -e * xp.sin(phase)]
        v = [sum(vprime[i] * float(self.E[i, c]) for i in range(3)) for c in range(3)]
        B = [sum(bprime[i] * float(self.E[i, c]) for i in range(3)) for c in range(3)]
        return dict(rho=one, v=v, p=self.p0 * one, B=B, psi=0.0 * one)


def _radius(x, c):
    """Euclidean distance of the points x[P, D] from the point c (no periodic wrap)."""
    xp = _xp(x)
    d = x - (c if xp is np else torch.as_tensor(c, dtype=x.dtype, device=x.device))
    return xp.sqrt((d * d).sum(axis=-1) if xp is np else (d * d).sum(dim=-1))


class OrszagTang:
    """Orszag-Tang vortex (2-D, gamma 5/3)."""

    def __call__(self, x):
        xp = _xp(x)
        tp = 2.0 * math.pi
        b0 = 1.0 / math.sqrt(4.0 * math.pi)
        X, Y = x[:, 0], x[:, 1]
        z = _const(xp, X, 0.0)
        return dict(rho=_const(xp, X, 25.0 / (36.0 * math.pi)), p=_const(xp, X, 5.0 / (12.0 * math.pi)),
                    v=[-xp.sin(tp * Y), xp.sin(tp * X), z], B=[-b0 * xp.sin(tp * Y), b0 * xp.sin(2 * tp * X), z],
                    psi=z)


class Rotor:
    """First rotor problem (2-D; the paper states no gamma for it, the runs
    here take 1.4, that of the problem's original definition)."""

    r0, r1, v0 = 0.1, 0.115, 2.0

    def __call__(self, x):
        xp = _xp(x)
        X, Y = x[:, 0], x[:, 1]
        r = _radius(x, np.array([0.5, 0.5]))
        one = _const(xp, X, 1.0)
        f = xp.where(r < self.r0, one, xp.where(r > self.r1, 0.0 * one, (self.r1 - r) / (self.r1 - self.r0)))
        w = self.v0 / self.r0 * f
        z = 0.0 * one
        return dict(rho=1.0 + 9.0 * f, p=one, v=[(0.5 - Y) * w, (X - 0.5) * w, z],
                    B=[5.0 / math.sqrt(4.0 * math.pi) * one, z, z], psi=z)


class Blast2D:
    """Strongly magnetised blast wave in 2-D (B at 45 degrees to the grid)."""

    def __init__(self, B0=1.0):
        self.B0 = B0

    def __call__(self, x):
        xp = _xp(x)
        one = _const(xp, x[:, 0], 1.0)
        r = _radius(x, np.array([0.5, 0.5]))
        b = self.B0 / math.sqrt(2.0)
        z = 0.0 * one
        return dict(rho=one, p=xp.where(r < 0.1, 10.0 * one, 0.1 * one), v=[z, z, z], B=[b * one, b * one, z],
                    psi=z)


class Blast3D:
    """Blast wave with pressure ratio 1e4 in a strong field (gamma 1.4); the
    centre is moved half a cell of an n^3 grid off the box centre."""

    def __init__(self, n):
        self.c = np.full(3, 0.5 + 0.5 / n)

    def __call__(self, x):
        xp = _xp(x)
        one = _const(xp, x[:, 0], 1.0)
        r = _radius(x, self.c)
        b = 100.0 / (math.sqrt(3.0) * math.sqrt(4.0 * math.pi))
        z = 0.0 * one
        return dict(rho=one, p=xp.where(r < 0.1, 1000.0 * one, 0.1 * one), v=[z, z, z], B=[b * one, b * one, b * one],
                    psi=z)


class Loop:
    """Field-loop advection on [-1,1]^2 (mesh box 2, points shifted by -1)."""

    A0, R0 = 1e-3, 0.3

    def __call__(self, x):
        xp = _xp(x)
        xs = x - 1.0
        one = _const(xp, x[:, 0], 1.0)
        r = _radius(xs, np.array([0.0, 0.0]))
        inside = r < self.R0
        rs = xp.where(inside, r, one)
        z = 0.0 * one
        bx = xp.where(inside, -self.A0 * xs[:, 1] / rs, z)
        by = xp.where(inside, self.A0 * xs[:, 0] / rs, z)
        return dict(rho=one, p=one, v=[2.0 * one, one, z], B=[bx, by, z], psi=z)


def config_field(cfg, replicate=0):
    """Seeded field of a benchmark configuration (seed = 1000 cfg + replicate)."""
    seed = 1000 * cfg + replicate
    if cfg == 0:
        return Smooth(seed, 2)
    if cfg == 1:
        return Smooth(seed, 3)
    if cfg in (2, 4):
        return Blast(seed)
    if cfg == 3:
        return Peaks(seed)
    raise ValueError(cfg)


# ---------------------------------------------------------------------------
# octree leaves of the Gaussian-peak workload (mesh input, no scheme arithmetic)


def _morton_keys(level, ijk, lmax):
    """Z-order keys of leaves (level, ijk[:, 3]) on the finest grid (int64)."""
    c = ijk.astype(np.int64) << (lmax - level.astype(np.int64))[:, None]
    key = np.zeros(len(level), dtype=np.int64)
    for b in range(20):
        for a in range(3):
            key |= ((c[:, a] >> b) & 1) << (3 * b + a)
    return key


def _refine(level, ijk, flags):
    keep_l, keep_c = level[~flags], ijk[~flags]
    pl, pc = level[flags], ijk[flags]
    kids_l, kids_c = [], []
    for off in range(8):
        o = np.array([(off >> a) & 1 for a in range(3)], dtype=np.int64)
        kids_l.append(pl + 1)
        kids_c.append(2 * pc + o)
    return (np.concatenate([keep_l] + kids_l), np.concatenate([keep_c] + kids_c))


def peaks_leaves(peaks, n0=64, r1=0.14, r2=0.10):
    """Leaves (level[int8], ijk[int32, 3]) of the octree of the Gaussian-peak
    workload on [0,1]^3: base n0^3 cells refined where the cell centre is
    within r1 of a peak, their children again within r2; level-0 cells that
    touch a level-2 cell are refined (2:1 balance across faces); Morton
    order."""
    g = np.stack(np.meshgrid(np.arange(n0), np.arange(n0), np.arange(n0), indexing="ij"), -1).reshape(-1, 3)
    ijk = g[:, ::-1].astype(np.int64)   # x fastest
    level = np.zeros(len(ijk), dtype=np.int64)

    def centers(l, c):
        h = 1.0 / (n0 << l)
        return (c + 0.5) * h[:, None]

    level, ijk = _refine(level, ijk, peaks.refine_flags(centers(level, ijk), r1))
    f = peaks.refine_flags(centers(level, ijk), r2) & (level == 1)
    level, ijk = _refine(level, ijk, f)
    # 2:1 balance: a level-0 leaf must not touch a level-2 leaf
    for _ in range(4):
        l2 = ijk[level == 2] // 2          # level-1 parents of level-2 leaves
        n1 = n0 * 2
        nb = []
        for a in range(3):
            for s in (-1, 1):
                q = l2.copy()
                q[:, a] = (q[:, a] + s) % n1
                nb.append(q)
        nb = np.unique(np.concatenate(nb) // 2, axis=0)  # level-0 regions adjacent to refined level-1 cells
        key = lambda c: (c[:, 0] * n0 + c[:, 1]) * n0 + c[:, 2]
        is0 = level == 0
        bad = np.zeros(len(level), dtype=bool)
        bad[is0] = np.isin(key(ijk[is0]), key(nb))
        if not bad.any():
            break
        level, ijk = _refine(level, ijk, bad)
    order = np.argsort(_morton_keys(level, ijk, int(level.max())), kind="stable")
    return level[order].astype(np.int8), ijk[order].astype(np.int32)
