"""GPU parity of the limiters (TVB characteristic / componentwise slope
limiter and the FP64 positivity limiter) against the oracle, standalone and
inside SSP-RK3 steps, on seeded blast-wave inputs (8 over-pressured spheres,
the shocked configuration of the benchmark suite) at small sizes."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import dg, limiters
from parity_util import block_rel_max, make_pair, rel_l1, to_cells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G = 5.0 / 3.0


def _announce(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("D,d,n,lim", [(3, 2, 6, 7), (3, 3, 5, 7), (3, 2, 6, 5), (2, 2, 16, 7), (2, 1, 24, 7),
                                       (3, 3, 5, 4)])
def test_limit_matches_oracle(D, d, n, lim):
    _announce("limit", D, d, n, lim)
    field = wl.Blast(2000) if D == 3 else wl.Blast(2001)
    if D == 2:
        base = field
        field = lambda x, base=base: base(np.concatenate([x, np.full((x.shape[0], 1), 0.5)], 1)
                                          if isinstance(x, np.ndarray) else
                                          torch.cat([x, torch.full_like(x[:, :1], 0.5)], 1))
    gpu, wg, orc, wo = make_pair(D, d, n, dg.GLM, field=field, limiter=lim)
    st_o = {}
    olim = limiters.make_stage_limiter(orc, lim, stats=st_o)
    wo2 = olim(wo)
    st_g = gpu.limit(wg, stats=True)
    wg2 = to_cells(wg, orc.mesh.ncells)
    assert st_g["n_tvb_triggered"] == st_o.get("n_tvb", 0)
    assert st_g["n_pos_scaled"] == st_o.get("n_pos_scaled", 0)
    assert st_g["n_floor"] == st_o.get("n_floor", 0)
    if lim & 1:
        assert st_o["n_tvb"] > 0
    err = block_rel_max(wg2, wo2, orc)
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("D,d,n,lim", [(3, 2, 6, 7), (3, 3, 5, 7), (2, 2, 16, 7)])
def test_limited_steps_match_oracle(D, d, n, lim):
    _announce("limited steps", D, d, n, lim)
    field = wl.Blast(2000)
    if D == 2:
        base = field
        field = lambda x, base=base: base(np.concatenate([x, np.full((x.shape[0], 1), 0.5)], 1)
                                          if isinstance(x, np.ndarray) else
                                          torch.cat([x, torch.full_like(x[:, :1], 0.5)], 1))
    gpu, wg, orc, wo = make_pair(D, d, n, dg.GLM, field=field, limiter=lim)
    olim = limiters.make_stage_limiter(orc, lim)
    wo = olim(wo)
    gpu.limit(wg)
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo, limiter=olim)
    gpu.step(wg, 3)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=ch)
    assert np.all(err < 1e-12), err


def test_limited_steps_fp32_error_stated():
    """FP32 path with limiters (FP64 decisions and positivity): rel-L1 vs the
    FP64 oracle after 3 steps on the blast input stays below 1e-5."""
    _announce("limited fp32")
    gpu, wg, orc, wo = make_pair(3, 3, 5, dg.GLM, precision=1, field=wl.Blast(2000), limiter=7)
    olim = limiters.make_stage_limiter(orc, 7)
    wo = olim(wo)
    gpu.limit(wg)
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo, limiter=olim)
    gpu.step(wg, 3)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=ch)
    print("fp32 limited rel-L1", err, flush=True)
    assert np.all(err < 1e-5), err


def _blast(D):
    """The 3-D blast input, or its z = 0.5 slice in 2-D."""
    if D == 3:
        return wl.Blast(2000)
    base = wl.Blast(2001)
    return lambda x: base(np.concatenate([x, np.full((x.shape[0], 1), 0.5)], 1) if isinstance(x, np.ndarray) else
                          torch.cat([x, torch.full_like(x[:, :1], 0.5)], 1))


@pytest.mark.parametrize("D,d,n,lim", [(3, 2, 8, 7), (3, 2, 8, 5), (3, 1, 8, 7), (3, 3, 6, 7), (3, 2, 8, 1),
                                       (2, 2, 20, 7), (2, 3, 16, 7), (2, 1, 24, 5)])
def test_powell_limit_matches_oracle(D, d, n, lim):
    """Powell scheme with the LDF field (Sec. 4.2.4): 8-wave characteristic
    (or componentwise) TVB decisions, limited Legendre slopes, the
    divergence-free re-projected field and positivity against the oracle."""
    _announce("powell limit", D, d, n, lim)
    gpu, wg, orc, wo = make_pair(D, d, n, dg.POWELL, field=_blast(D), limiter=lim)
    st_o = {}
    wo2 = limiters.make_stage_limiter(orc, lim, stats=st_o)(wo)
    st_g = gpu.limit(wg, stats=True)
    wg2 = to_cells(wg, orc.mesh.ncells)
    assert st_o["n_tvb"] > 0
    assert st_g["n_tvb_triggered"] == st_o["n_tvb"]
    assert st_g["n_pos_scaled"] == st_o.get("n_pos_scaled", 0)
    err = block_rel_max(wg2, wo2, orc)
    assert np.all(err < 1e-12), err
    # every troubled cell carries a divergence-free linear field (positivity
    # scales it about its mean, which keeps it so)
    _, troubled = limiters.slope_limit(orc, wo, characteristic=bool(lim & 2))
    Pm, Pl = limiters.ldf_moments(orc)
    nl = len(orc.leg_vars) * orc.n
    S = np.einsum("cbl,kl->kcb", Pl, wg2[troubled, nl:])
    tr = np.abs(np.trace(S, axis1=1, axis2=2))
    assert np.all(tr < 1e-12 * np.maximum(1.0, np.abs(S).max(axis=(1, 2)))), tr.max()


@pytest.mark.parametrize("D,d,n", [(3, 2, 8), (2, 2, 20)])
def test_powell_limited_steps_match_oracle(D, d, n):
    _announce("powell limited steps", D, d, n)
    gpu, wg, orc, wo = make_pair(D, d, n, dg.POWELL, field=_blast(D), limiter=7)
    olim = limiters.make_stage_limiter(orc, 7)
    wo = olim(wo)
    gpu.limit(wg)
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo, limiter=olim)
    gpu.step(wg, 3)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo)
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("D,divb", [(2, dg.GLM), (2, dg.POWELL), (3, dg.GLM), (3, dg.POWELL)])
def test_limit_at_the_pressure_floor_in_a_strong_field_matches_oracle(D, divb):
    """Cells whose mean pressure is ten times the floor in a field of
    |B|^2/p ~ 1e14: the characteristic matrices there are not used
    (componentwise limiting; the cells' condition number would exceed 1e13);
    decisions, states and counts match the oracle, and every weight stays
    finite.  (Exactly at the floor the floor decision itself would rest on
    the rounding of E - |B|^2/2 ~ 4e-14.)"""
    from paper_1806_02343_amd import DG
    _announce("floor strong field", D, divb)
    n = 12 if D == 2 else 10
    b = 100.0 / np.sqrt(3.0) / np.sqrt(4.0 * np.pi)

    def prim(x):
        # pressure constant per cell (by the cell centre's radius), so that a
        # cell mean is either at the floor or well conditioned (|B|^2/p of
        # about 8e2 and 1e-1); density varies smoothly, v = 0
        rc = np.sqrt((((np.floor(x * n) + 0.5) / n - 0.5) ** 2).sum(axis=1))
        one = np.ones(x.shape[0])
        p = np.where(rc < 0.15, 1000.0, np.where(rc < 0.4, 1e-11, 1.0)) * one
        rho = 1.0 + 0.9 * np.sin(6 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
        return dict(rho=rho, v=[0 * one, 0 * one, 0 * one], p=p, B=[b * one, b * one, b * one], psi=0 * one)
    orc = dg.DG(dg.Mesh.uniform(D, n), 2, divb=divb, gamma=1.4)
    wo = orc.project(dg.conserved_field(prim, 1.4, orc.nvar))
    means = orc.cell_means(wo)
    low = [not limiters.char_usable(means[:, k], 1.4) for k in range(orc.mesh.ncells)]
    assert any(low) and not all(low)
    for lim in (3, 7):
        gpu = DG(D, 2, n, divb=divb, limiter=lim, gamma=1.4)
        wg = torch.as_tensor(orc.to_abi(wo, gpu.ld), device="cuda")
        st_o = {}
        wo2 = limiters.make_stage_limiter(orc, lim, stats=st_o)(wo)
        st_g = gpu.limit(wg, stats=True)
        wg2 = to_cells(wg, orc.mesh.ncells)
        assert np.all(np.isfinite(wg2))
        assert st_g["n_tvb_triggered"] == st_o["n_tvb"] > 0
        assert st_g["n_pos_scaled"] == st_o.get("n_pos_scaled", 0)
        err = block_rel_max(wg2, wo2, orc)
        assert np.all(err < 1e-12), (lim, err)


@pytest.mark.parametrize("D,d,precision", [(3, 3, 0), (3, 2, 0), (3, 3, 1), (2, 3, 0)])
def test_positivity_near_floors_matches_oracle(D, d, precision):
    """Positivity limiter on states built around the floors, in tiles of 16
    cells: small higher modes (every point far above the floors), a spread of
    amplitudes (some cells with points below a floor, some just above), and
    large ones (nearly every cell scaled), in density and in energy.  Decisions,
    counts and states match the oracle, including on tiles the GPU path
    screens out from the means and mode magnitudes without evaluating them.
    FP64 within 1e-12 block-relative; FP32 within 1e-6 (the scaled modes are
    rounded to FP32)."""
    _announce("positivity near floors", D, d, precision)
    n = 8 if D == 3 else 24
    gpu, wg, orc, wo = make_pair(D, d, n, dg.GLM, limiter=4, precision=precision)
    rng = np.random.default_rng(700 + 10 * D + d)
    C, N = orc.mesh.ncells, orc.n
    tile = np.arange(C) // 16
    amp = np.where(tile % 3 == 0, 1e-3, np.where(tile % 3 == 1, rng.uniform(0.05, 0.6, C), rng.uniform(0.4, 1.0, C)))
    w = np.zeros((C, orc.nmodes))
    for v in range(9):
        w[:, v * N + 1:(v + 1) * N] = rng.normal(size=(C, N - 1)) * (amp / np.sqrt(N - 1))[:, None]
    w[:, 0] = 1.0
    for v in (1, 2, 3, 5, 6, 7, 8):
        w[:, v * N] = rng.uniform(-0.3, 0.3, C)
    ke = 0.5 * sum(w[:, v * N] ** 2 for v in (1, 2, 3))
    me = 0.5 * sum(w[:, v * N] ** 2 for v in (5, 6, 7))
    w[:, 4 * N] = 0.3 / (G - 1.0) + ke + me
    w[:, 4 * N + 1:5 * N] *= w[:, 4 * N][:, None]
    if precision == 1:
        w = w.astype(np.float32).astype(np.float64)
    wg[:, :C] = torch.as_tensor(w.T.copy(), dtype=wg.dtype, device=wg.device)
    torch.cuda.synchronize()
    wo2, st_o = limiters.positivity(orc, w)
    st_g = gpu.limit(wg, stats=True)
    scaled = np.any(wo2 != w, axis=1)
    assert not scaled[tile % 3 == 0].any() and scaled[tile % 3 == 2].mean() > 0.9
    assert 0 < scaled[tile % 3 == 1].sum() < (tile % 3 == 1).sum()  # mixed tiles hold both kinds
    assert st_g["n_pos_scaled"] == st_o["n_pos_scaled"]
    assert st_g["n_floor"] == st_o["n_floor"]
    err = block_rel_max(to_cells(wg, C), wo2, orc)
    assert np.all(err < (1e-12 if precision == 0 else 1e-6)), err
