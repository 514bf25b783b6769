"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs (projection, right-hand side, time step, SSP-RK3 steps).
FP64 must agree to 1e-12 relative; the FP32 path to 1e-5 relative L1."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import dg
from parity_util import block_rel_max, make_pair, rel_l1, to_cells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (D, d, n, divb): 2-D config-0 shape, 3-D GLM and Powell/LDF with ragged tiles
CASES = [
    (2, 1, 32, dg.GLM),
    (2, 2, 12, dg.GLM),
    (2, 3, 10, dg.GLM),
    (3, 1, 7, dg.GLM),
    (3, 2, 6, dg.GLM),
    (3, 3, 5, dg.GLM),
    (3, 1, 5, dg.POWELL),
    (3, 2, 6, dg.POWELL),
    (2, 1, 16, dg.POWELL),
    (2, 2, 12, dg.POWELL),
    (2, 3, 9, dg.POWELL),
]


def ids(c):
    return f"D{c[0]}d{c[1]}n{c[2]}{'glm' if c[3] == dg.GLM else 'powell'}"


def _announce(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_projection_matches_oracle(case):
    D, d, n, divb = case
    _announce("projection", case)
    gpu, wg, orc, wo = make_pair(D, d, n, divb)
    wgc = to_cells(wg, orc.mesh.ncells)
    assert np.all(block_rel_max(wgc, wo, orc) < 1e-13)
    # padding columns stay zero
    assert float(wg[:, orc.mesh.ncells:].abs().max() if wg.shape[1] > orc.mesh.ncells else 0.0) == 0.0


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_rhs_matches_oracle(case):
    D, d, n, divb = case
    _announce("rhs", case)
    gpu, wg, orc, wo = make_pair(D, d, n, divb)
    dt, ch, kappa = orc.timestep(wo)
    if divb == dg.GLM:
        # give psi a nonzero state so the GLM fluxes and damping are exercised
        rng = np.random.default_rng(5)
        wo[:, 8 * orc.n:] = 0.05 * rng.normal(size=(orc.mesh.ncells, orc.n))
        wg[:, :orc.mesh.ncells] = torch.as_tensor(wo.T, device="cuda")
    r_o = orc.rhs(wo, ch, kappa)
    out = gpu.empty_state()
    gpu.rhs(wg, out, ch, kappa)
    torch.cuda.synchronize()
    r_g = to_cells(out, orc.mesh.ncells)
    err = block_rel_max(r_g, r_o, orc)
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("case", [(2, 1, 32, dg.GLM), (3, 3, 5, dg.GLM), (3, 2, 6, dg.POWELL), (2, 3, 9, dg.POWELL)],
                         ids=ids)
@pytest.mark.parametrize("prec", [0, 1])
def test_nodal_values_match_oracle(case, prec):
    """dg_nodal: the state at the (d+3)^D points of the projection rule
    against the oracle's evaluation of the same weights, all cells and a
    sub-range."""
    D, d, n, divb = case
    _announce("nodal", case, prec)
    gpu, wg, orc, wo = make_pair(D, d, n, divb, precision=prec)
    wc = to_cells(wg, orc.mesh.ncells)
    xi = gpu.proj_points()
    U = orc.nodal(wc, xi=xi)                                # [var, cell, point]
    out = gpu.nodal(wg).cpu().numpy()                       # [var, point, cell]
    assert out.shape == (orc.nvar, xi.shape[0], orc.mesh.ncells)
    scale = np.abs(U).max(axis=(1, 2))
    err = np.abs(out.transpose(0, 2, 1) - U).max(axis=(1, 2)) / np.maximum(scale, 1e-3 * scale.max())
    assert np.all(err < 1e-13), err
    c0, nc = 7, orc.mesh.ncells // 3
    sub = gpu.nodal(wg, c0, nc).cpu().numpy()
    assert np.array_equal(sub, out[:, :, c0:c0 + nc])


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_timestep_matches_oracle(case):
    D, d, n, divb = case
    _announce("dt", case)
    gpu, wg, orc, wo = make_pair(D, d, n, divb)
    dto, cho, ko = orc.timestep(wo)
    dtg, chg, kg = gpu.dt(wg)
    assert abs(dtg - dto) <= 1e-13 * dto
    assert abs(chg - cho) <= 1e-13 * max(cho, 1e-300)
    assert abs(kg - ko) <= 1e-13 * max(ko, 1e-300)


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_steps_match_oracle_fp64(case):
    D, d, n, divb = case
    nsteps = 10 if D == 2 else 3
    _announce("steps fp64", case, nsteps)
    gpu, wg, orc, wo = make_pair(D, d, n, divb)
    t_o = 0.0
    for _ in range(nsteps):
        wo, dt, ch, k = orc.step(wo)
        t_o += dt
    t_g = gpu.step(wg, nsteps)
    assert abs(t_g - t_o) <= 1e-12 * t_o
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=max(ch, 1.0))
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_steps_match_oracle_fp32(case):
    D, d, n, divb = case
    nsteps = 10 if D == 2 else 3
    _announce("steps fp32", case, nsteps)
    gpu, wg, orc, wo = make_pair(D, d, n, divb, precision=1)
    for _ in range(nsteps):
        wo, dt, ch, k = orc.step(wo)
    gpu.step(wg, nsteps)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=max(ch, 1.0))
    assert np.all(err < 1e-5), err


def test_config0_ten_steps_rel_l1():
    """Config 0: 2-D 32x32, d = 1, GLM, smooth seeded IC, 10 SSP-RK3 steps at CFL 0.3."""
    _announce("config0")
    field = wl.config_field(0)
    gpu, wg, orc, wo = make_pair(2, 1, 32, dg.GLM, field=field)
    for _ in range(10):
        wo, dt, ch, k = orc.step(wo)
    gpu.step(wg, 10)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=ch)
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("case", [(3, 3, 5, dg.GLM), (3, 2, 6, dg.GLM), (2, 2, 12, dg.GLM)], ids=ids)
def test_matrix_core_schedule_steps_fp64(case):
    """Three SSP-RK3 steps with the matrix-core cell and face kernels (schedule
    4 + 16) against the oracle at 1e-12."""
    D, d, n, divb = case
    _announce("mfma steps", case)
    gpu, wg, orc, wo = make_pair(D, d, n, divb)
    gpu.autotune(wg, variant=4 + 16)
    dt_g, ch_g, _ = gpu.dt(wg)
    dt_o, ch_o, _ = orc.timestep(wo)
    assert abs(dt_g - dt_o) <= 1e-12 * dt_o and abs(ch_g - ch_o) <= 1e-12 * ch_o
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo)
    gpu.step(wg, 3)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=ch)
    assert np.all(err < 1e-12), err


def test_step_is_deterministic():
    _announce("determinism")
    gpu, wg, orc, wo = make_pair(3, 2, 6, dg.GLM)
    w2 = wg.clone()
    gpu.step(wg, 2)
    gpu.step(w2, 2)
    assert torch.equal(wg, w2)


VARIANT_CASES = [(3, 2, 6, dg.GLM), (3, 3, 5, dg.GLM), (3, 1, 7, dg.GLM), (3, 2, 6, dg.POWELL), (2, 2, 12, dg.GLM),
                 (2, 3, 9, dg.GLM), (2, 1, 11, dg.GLM), (2, 2, 12, dg.POWELL), (2, 3, 9, dg.POWELL)]


@pytest.mark.parametrize("case", VARIANT_CASES, ids=ids)
def test_every_cell_tile_variant_matches_oracle(case):
    """Each tile shape the autotuner may pick gives the same right-hand side."""
    D, d, n, divb = case
    _announce("variants", case)
    gpu, wg, orc, wo = make_pair(D, d, n, divb)
    dt, ch, kappa = orc.timestep(wo)
    r_o = orc.rhs(wo, ch, kappa)
    ran = 0
    for v in [c + 16 * f for f in range(4) for c in range(10)]:  # cell variant + 16 x face variant
        try:
            gpu.autotune(wg, variant=v)
        except Exception:
            continue
        out = gpu.empty_state()
        gpu.rhs(wg, out, ch, kappa)
        torch.cuda.synchronize()
        err = block_rel_max(to_cells(out, orc.mesh.ncells), r_o, orc)
        assert np.all(err < 1e-12), (v, err)
        ran += 1
    assert ran >= (8 if divb == dg.GLM else 2)
    chosen = gpu.autotune(wg)
    assert 0 <= (chosen & 15) < 10 and 0 <= (chosen >> 4) < 4


@pytest.mark.parametrize("case", [c for c in VARIANT_CASES if c[3] == dg.GLM], ids=ids)
def test_every_cell_variant_fp32(case):
    """FP32 right-hand sides of every cell-kernel variant (LDS-tiled and
    matrix-core) against the oracle, block-relative error below 5e-4: FP32
    rounding (2^-24) of about 3 x 10^2 accumulated terms per mode, times the
    cancellation between the volume and surface terms of a smooth state
    (up to ~10 for the psi block, whose right-hand side is the small
    difference of c_h^2 B terms), gives up to ~1e-4 depending on the order
    of accumulation, which differs between the variants."""
    D, d, n, divb = case
    _announce("variants fp32", case)
    gpu, wg, orc, wo = make_pair(D, d, n, divb, precision=1)
    dt, ch, kappa = orc.timestep(wo)
    r_o = orc.rhs(wo, ch, kappa)
    ran = 0
    for v in [c + 16 * f for f in range(4) for c in range(10)]:
        try:
            gpu.autotune(wg, variant=v)
        except Exception:
            continue
        out = gpu.empty_state()
        gpu.rhs(wg, out, ch, kappa)
        torch.cuda.synchronize()
        err = block_rel_max(to_cells(out, orc.mesh.ncells), r_o, orc)
        assert np.all(err < 5e-4), (v, err)
        if (v & 15) >= 4 and D == 3:
            # matrix-core kernels (FP32 deviation form): the background flux
            # is handled in FP64, leaving FP32 rounding of the deviations
            assert np.all(err < 2e-5), (v, err)
        ran += 1
    assert ran >= 8


def test_schedule_pairs_face_flux_layouts():
    """On uniform GLM grids the LDS kernels (cell 0-3, face 0) exchange face-point
    fluxes and the matrix-core kernels (cell 4-9, face 1-3) face moments: a
    schedule that pairs the two is refused, every compatible pair matches the
    oracle, and the autotuner keeps a compatible pair."""
    from paper_1806_02343_amd.binding import DGError
    _announce("schedule layouts")
    gpu, wg, orc, wo = make_pair(3, 2, 6, dg.GLM)
    dt, ch, kappa = orc.timestep(wo)
    r_o = orc.rhs(wo, ch, kappa)
    for v in (0 + 16 * 1, 3 + 16 * 2, 4 + 16 * 0, 9 + 16 * 0):
        with pytest.raises(DGError):
            gpu.autotune(wg, variant=v)
    lds = []
    for c in range(4):  # the LDS tile shapes built for this configuration
        try:
            gpu.autotune(wg, variant=c)
            lds.append(c)
        except DGError:
            pass
    assert lds
    for v in (lds[0], 4 + 16 * 1, 8 + 16 * 3):
        gpu.autotune(wg, variant=v)
        out = gpu.empty_state()
        gpu.rhs(wg, out, ch, kappa)
        torch.cuda.synchronize()
        err = block_rel_max(to_cells(out, orc.mesh.ncells), r_o, orc)
        assert np.all(err < 1e-12), (v, err)
    chosen = gpu.autotune(wg)
    assert ((chosen >> 4) >= 1) == ((chosen & 15) >= 4), chosen


@pytest.mark.parametrize("fv", [0, 1])
@pytest.mark.parametrize("D,d,n", [(3, 2, 6), (2, 2, 12)])
def test_powell_dt_cap_binds_matches_oracle(D, d, n, fv):
    """Powell time-step cap (eq. powell_dt with |div B|_K from the face jumps of
    eq. divb-cell) on a state with O(0.1) normal-field jumps at every face and
    a small eta, so that the cap and not eq. cfl sets the step: dg_dt and two
    SSP-RK3 steps against the oracle, with the LDS-staged face kernel and
    signal speeds (face variant 0) and with the matrix-core ones (1)."""
    from paper_1806_02343_amd import DG
    _announce("powell cap", D, d, n, fv)
    eta = 1e-6
    orc = dg.DG(dg.Mesh.uniform(D, n), d, divb=dg.POWELL, powell_eta=eta)
    rng = np.random.default_rng(77)
    wo = orc.project(dg.conserved_field(wl.Smooth(1000 * D + d, D), 5.0 / 3.0, orc.nvar))
    nl = len(orc.leg_vars) * orc.n
    wo[:, :nl] += 0.02 * rng.normal(size=(orc.mesh.ncells, nl)) * (np.arange(nl) % orc.n != 0)
    wo[:, nl:] += 0.05 * rng.normal(size=(orc.mesh.ncells, orc.nldf))
    gpu = DG(D, d, n, divb=dg.POWELL, powell_eta=eta)
    wg = torch.as_tensor(orc.to_abi(wo, gpu.ld), device="cuda")
    if fv:
        gpu.autotune(wg, variant=8 + 16 * fv)
    dt_o, _, _ = orc.timestep(wo)
    dt_cfl = dg.DG(dg.Mesh.uniform(D, n), d, divb=dg.POWELL).timestep(wo)[0]
    assert dt_o < 0.2 * dt_cfl          # the cap binds by a wide margin
    dt_g, _, _ = gpu.dt(wg)
    assert abs(dt_g - dt_o) <= 1e-13 * dt_o
    t_o = 0.0
    for _ in range(2):
        wo, dt, _, _ = orc.step(wo)
        t_o += dt
    t_g = gpu.step(wg, 2)
    assert abs(t_g - t_o) <= 1e-12 * t_o
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo)
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("case", [(3, 2, 6, dg.POWELL), (3, 1, 7, dg.POWELL), (3, 3, 5, dg.POWELL),
                                  (2, 2, 12, dg.POWELL), (2, 3, 9, dg.POWELL)], ids=ids)
@pytest.mark.parametrize("cv", [6, 8])
def test_powell_matrix_core_schedule_steps_fp64(case, cv):
    """The Powell scheme with the matrix-core face kernel (face variant 1),
    whose time step evaluates the signal speeds on the matrix cores and takes
    the cap from the jumps the first stage's face launch wrote, and the
    persistent (6) or plain (8) matrix-core cell kernel: dg_dt and three
    SSP-RK3 steps against the oracle at 1e-12."""
    D, d, n, divb = case
    _announce("powell mfma steps", case, cv)
    gpu, wg, orc, wo = make_pair(D, d, n, divb)
    gpu.autotune(wg, variant=cv + 16)
    dt_g, _, _ = gpu.dt(wg)
    dt_o, _, _ = orc.timestep(wo)
    assert abs(dt_g - dt_o) <= 1e-12 * dt_o
    t_o = 0.0
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo)
        t_o += dt
    t_g = gpu.step(wg, 3)
    assert abs(t_g - t_o) <= 1e-12 * t_o
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=max(ch, 1.0))
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("case", [(3, 3, 5, dg.GLM), (3, 2, 6, dg.GLM), (2, 1, 11, dg.GLM), (2, 3, 9, dg.GLM)],
                         ids=ids)
def test_fp32_matrix_core_path_preserves_a_uniform_state(case):
    """FP32 deviation form of the matrix-core kernels: the products act on the
    modes above the cell mean and on fluxes minus a per-face reference flux
    (the mean state's flux handled in FP64), so a uniform state, whose exact
    right-hand side is zero, gives zero up to FP64 rounding; the FP32 products
    of the full fluxes (LDS kernels) leave ~1e-5 of the background flux."""
    D, d, n, divb = case
    _announce("fp32 free stream", case)
    gpu, wg, orc, wo = make_pair(D, d, n, divb, precision=1)
    u = np.array([1.3, 0.2, -0.1, 0.3, 4.0, 0.7, -0.4, 0.5, 0.25])
    wu = np.zeros_like(wo)
    for k in range(9):
        wu[:, k * orc.n] = u[k]
    wgu = torch.as_tensor(orc.to_abi(wu, gpu.ld), dtype=torch.float32, device="cuda")
    for v in (4 + 16, 6 + 32, 8 + 48):
        gpu.autotune(wgu, variant=v)
        out = gpu.empty_state()
        gpu.rhs(wgu, out, 2.0, 0.5)
        torch.cuda.synchronize()
        r = out[:, :orc.mesh.ncells].double().cpu().numpy()
        r[8 * orc.n] += 0.5 * 0.25          # the GLM damping of psi is the only nonzero term
        assert np.abs(r).max() < 1e-10, (v, np.abs(r).max())


RK_CASES = [(2, 1, 16, dg.GLM, 1), (2, 2, 12, dg.GLM, 2), (3, 3, 5, dg.GLM, 5), (3, 2, 6, dg.POWELL, 5),
            (3, 1, 7, dg.GLM, 2), (3, 2, 5, dg.POWELL, 1)]


@pytest.mark.parametrize("case", RK_CASES, ids=lambda c: ids(c[:4]) + f"rk{c[4]}")
def test_ssp_rk_schemes_match_oracle(case):
    """Forward Euler, SSP-RK2 and the five-stage fourth-order SSP scheme
    (Sec. 3.6: order 1-4) against the oracle's Shu-Osher steps, FP64 to 1e-12."""
    D, d, n, divb, rk = case
    nsteps = 4
    _announce("rk", case)
    gpu, wg, orc, wo = make_pair(D, d, n, divb, rk_stages=rk)
    t_o = 0.0
    for _ in range(nsteps):
        wo, dt, ch, k = orc.step(wo, rk=rk)
        t_o += dt
    t_g = gpu.step(wg, nsteps)
    assert abs(t_g - t_o) <= 1e-12 * t_o
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=max(ch, 1.0))
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("rk", [2, 5])
def test_ssp_rk_with_limiters_match_oracle(rk):
    """The limited blast with SSP-RK2 and SSP-RK(5,4): the limiters after every
    stage, including the fourth stage of the (5,4) scheme, whose unlimited
    state also enters the final combination."""
    from oracle import limiters
    _announce("rk limited", rk)
    gpu, wg, orc, wo = make_pair(3, 2, 6, dg.GLM, field=wl.Blast(2000), limiter=7, rk_stages=rk)
    olim = limiters.make_stage_limiter(orc, 7)
    wo = olim(wo)
    gpu.limit(wg)
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo, limiter=olim, rk=rk)
    gpu.step(wg, 3)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=ch)
    assert np.all(err < 1e-12), err


def test_ssp_rk4_fp32_matches_oracle():
    _announce("rk5 fp32")
    gpu, wg, orc, wo = make_pair(3, 2, 6, dg.GLM, precision=1, rk_stages=5)
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo, rk=5)
    gpu.step(wg, 3)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=max(ch, 1.0))
    assert np.all(err < 1e-5), err


@pytest.mark.parametrize("case", [(3, 1, 5, dg.POWELL), (3, 2, 6, dg.POWELL), (3, 3, 4, dg.POWELL),
                                  (2, 2, 10, dg.POWELL)], ids=ids)
def test_powell_interpolated_q_matches_oracle(case):
    """Powell face term with the interpolated q-dagger (eq. powellq-interp,
    HLLD interface state) on a state with normal-field jumps at every face:
    the right-hand side of every cell-kernel variant and three SSP-RK3 steps
    against the oracle, FP64 to 1e-12."""
    from paper_1806_02343_amd import DG
    D, d, n, divb = case
    _announce("powell interp", case)
    orc = dg.DG(dg.Mesh.uniform(D, n), d, divb=dg.POWELL, powell_q="interp")
    rng = np.random.default_rng(88 + d)
    wo = orc.project(dg.conserved_field(wl.Smooth(1000 * D + d, D), 5.0 / 3.0, orc.nvar))
    nl = len(orc.leg_vars) * orc.n
    wo[:, :nl] += 0.01 * rng.normal(size=(orc.mesh.ncells, nl)) * (np.arange(nl) % orc.n != 0)
    wo[:, nl:] += 0.03 * rng.normal(size=(orc.mesh.ncells, orc.nldf))
    gpu = DG(D, d, n, divb=dg.POWELL, powell_q=1)
    wg = torch.as_tensor(orc.to_abi(wo, gpu.ld), device="cuda")
    dt, ch, kappa = orc.timestep(wo)
    r_o = orc.rhs(wo, ch, kappa)
    ran = 0
    for v in [c + 16 * f for f in range(2) for c in range(10)]:   # cell variant + 16 x face variant
        try:
            gpu.autotune(wg, variant=v)
        except Exception:
            continue
        out = gpu.empty_state()
        gpu.rhs(wg, out, 0.0, 0.0)
        torch.cuda.synchronize()
        err = block_rel_max(to_cells(out, orc.mesh.ncells), r_o, orc)
        assert np.all(err < 1e-12), (v, err)
        ran += 1
    assert ran >= 4
    gpu.autotune(wg, variant=-1)
    t_o = 0.0
    for _ in range(3):
        wo, dt, _, _ = orc.step(wo)
        t_o += dt
    t_g = gpu.step(wg, 3)
    assert abs(t_g - t_o) <= 1e-12 * t_o
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo)
    assert np.all(err < 1e-12), err
