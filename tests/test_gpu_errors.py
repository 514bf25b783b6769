"""GPU tests of the error contract and of the positivity floors:

* cell-average floors that fire (negative mean density, negative mean
  pressure; Sec. 4.3): counts, injected mass and energy and the limited state
  against the oracle, on the matrix-core (GLM) and LDS-tiled (Powell)
  positivity kernels, FP64 and FP32; the tallies are bitwise reproducible;
* a non-finite weight makes dg_dt, dg_limit (with stats) and dg_step (with a
  time pointer) return DG_ENONFINITE, and the handle works again on a clean
  state;
* a fixed c_h below twice the largest signal speed (the runtime check of
  Sec. 4.1.5) gives the warning-class DG_ECH with valid outputs, counted in
  dg_limit_stats.n_ch_violation.

Every state is written from the host; every kernel runs to completion."""
import math
import sys
import warnings

import numpy as np
import pytest

import workloads as wl
from oracle import dg, limiters
from parity_util import block_rel_max, make_pair, to_cells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G = 5.0 / 3.0


def _announce(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


def _floored_state(orc, wo, seed):
    """Cells with a negative mean density (momentum zeroed), cells with a
    negative mean pressure, the rest untouched."""
    rng = np.random.default_rng(seed)
    w = wo.copy()
    C, N = orc.mesh.ncells, orc.n
    idx = rng.permutation(C)
    A, Bc = idx[:C // 9], idx[C // 9:C // 4]
    w[A, 0] = -rng.uniform(0.005, 0.05, A.size)
    for v in (1, 2, 3):
        w[A, v * N:(v + 1) * N] = 0.0
    Ub = orc.cell_means(w)
    ke = 0.5 * (Ub[1] ** 2 + Ub[2] ** 2 + Ub[3] ** 2) / Ub[0]
    me = 0.5 * (Ub[5] ** 2 + Ub[6] ** 2 + Ub[7] ** 2)
    w[Bc, 4 * N] = ke[Bc] + me[Bc] - rng.uniform(0.001, 0.02, Bc.size) / (G - 1.0)
    return w, A, Bc


@pytest.mark.parametrize("D,d,n,divb,prec", [(3, 2, 6, dg.GLM, 0), (3, 3, 5, dg.GLM, 0), (3, 2, 6, dg.GLM, 1),
                                              (2, 2, 16, dg.GLM, 0), (3, 2, 6, dg.POWELL, 0),
                                              (3, 1, 5, dg.POWELL, 0)])
def test_floors_fire_and_tallies_match_oracle(D, d, n, divb, prec):
    _announce("floors", D, d, n, divb, prec)
    gpu, wg, orc, wo = make_pair(D, d, n, divb, limiter=4, precision=prec)
    w, A, Bc = _floored_state(orc, wo, 900 + 10 * D + d + divb)
    if prec == 1:
        w = w.astype(np.float32).astype(np.float64)
    C = orc.mesh.ncells
    w_in = torch.as_tensor(orc.to_abi(w, gpu.ld), dtype=wg.dtype, device="cuda")
    wo2, st_o = limiters.positivity(orc, w)
    runs = []
    for _ in range(2):
        wg2 = w_in.clone()
        runs.append((wg2, gpu.limit(wg2, stats=True)))
    (wg2, st_g), (wg3, st_g2) = runs
    # closed form of the density floor's injected mass: sum (eps - rho_bar) h^D
    vol = orc.mesh.h[0] ** D
    assert st_o["n_floor"] >= A.size + Bc.size
    assert math.isclose(st_o["injected_mass"], float(((1e-12 - w[A, 0]) * vol).sum()), rel_tol=1e-12)
    assert st_g["n_floor"] == st_o["n_floor"]
    assert st_g["n_pos_scaled"] == st_o["n_pos_scaled"]
    # FP32: a floored mean is stored rounded up to the next FP32 value (the
    # energy floor sits ~1e-12 above E - |m|^2/2rho - |B|^2/2, far below the
    # FP32 resolution of E ~ 2, 2.4e-7); the tally is what was stored, up to
    # one FP32 ulp of E per floored cell against de ~ 1e-3 vol
    tol = 1e-12 if prec == 0 else 5e-4
    assert math.isclose(st_g["injected_mass"], st_o["injected_mass"], rel_tol=tol)
    assert math.isclose(st_g["injected_energy"], st_o["injected_energy"], rel_tol=tol)
    # fixed-order sums: bitwise the same on a second run
    assert st_g2["injected_mass"] == st_g["injected_mass"]
    assert st_g2["injected_energy"] == st_g["injected_energy"]
    assert torch.equal(wg2, wg3)
    wgc = to_cells(wg2, C)
    err = block_rel_max(wgc, wo2, orc)
    # FP32: a floored cell keeps p_bar a few 1e-7 above the floor, so its
    # scaling factor is ~1e-6 where the oracle's is 0
    assert np.all(err < (1e-12 if prec == 0 else 5e-6)), err
    # every cell's mean now clears both floors as stored
    Ub = orc.cell_means(wgc)
    pb = (G - 1.0) * (Ub[4] - 0.5 * (Ub[1] ** 2 + Ub[2] ** 2 + Ub[3] ** 2) / Ub[0] - 0.5 * (Ub[5] ** 2 + Ub[6] ** 2 + Ub[7] ** 2))
    assert Ub[0].min() >= 1e-12 and pb.min() >= 1e-12 * (1 - 1e-3)


def test_floor_tallies_inside_steps_are_summed_per_call():
    """dg_limit twice on the same floored state: each call reports its own
    tallies (the slots are cleared by the fixed-order sum)."""
    _announce("floors twice")
    gpu, wg, orc, wo = make_pair(3, 2, 6, dg.GLM, limiter=4)
    w, A, Bc = _floored_state(orc, wo, 17)
    w_in = torch.as_tensor(orc.to_abi(w, gpu.ld), device="cuda")
    a = gpu.limit(w_in.clone(), stats=True)
    b = gpu.limit(w_in.clone(), stats=True)
    assert a["injected_mass"] > 0 and a == b


def _nan_at(wg, mode, cell):
    bad = wg.clone()
    bad[mode, cell] = float("nan")
    return bad


def test_nonfinite_state_is_reported_and_not_sticky():
    from paper_1806_02343_amd import DGError
    from paper_1806_02343_amd.binding import DG_ENONFINITE
    _announce("nonfinite")
    gpu, wg, orc, wo = make_pair(3, 2, 6, dg.GLM, limiter=7)
    N = orc.n
    gpu.limit(wg)
    clean = wg.clone()
    with pytest.raises(DGError) as e:
        gpu.dt(_nan_at(clean, 1 * N + 3, 17))          # momentum: the signal speed is NaN
    assert e.value.code == DG_ENONFINITE
    with pytest.raises(DGError) as e:
        gpu.limit(_nan_at(clean, 1 * N + 1, 40), stats=True)
    assert e.value.code == DG_ENONFINITE
    with pytest.raises(DGError) as e:
        gpu.step(_nan_at(clean, 2, 100), 1)            # density: spreads through the step
    assert e.value.code == DG_ENONFINITE
    # the handle reports a clean state as clean again
    dt, ch, kappa = gpu.dt(clean)
    assert dt > 0 and math.isfinite(dt)
    st = gpu.limit(clean.clone(), stats=True)
    assert st["n_ch_violation"] == 0
    assert gpu.step(clean.clone(), 1) > 0


def test_fixed_ch_below_twice_the_signal_speed_warns():
    from paper_1806_02343_amd import DG, DGWarning
    _announce("ch check")
    D, d, n = 3, 2, 6
    field = wl.Smooth(1000 * D + d, D)
    orc = dg.DG(dg.Mesh.uniform(D, n), d)
    wo = orc.project(dg.conserved_field(field, G, 9))
    smax = orc.max_signal(wo).max() / D                 # the signal speed c_h is compared with
    low, high = 1.5 * smax, 4.0 * smax
    for ch_fixed, warn in ((low, True), (high, False)):
        orc_f = dg.DG(dg.Mesh.uniform(D, n), d, glm_ch_fixed=ch_fixed)
        dt_o, ch_o, k_o = orc_f.timestep(wo)
        gpu = DG(D, d, n, glm_ch_fixed=ch_fixed, limiter=7)
        wg = gpu.empty_state()
        wg[:, :orc.mesh.ncells] = torch.as_tensor(wo.T.copy(), device="cuda")
        with warnings.catch_warnings(record=True) as rec:
            warnings.simplefilter("always")
            dt_g, ch_g, k_g = gpu.dt(wg)
            st = gpu.limit(wg.clone(), stats=True)
            gpu.step(wg.clone(), 2)
        got = [r for r in rec if issubclass(r.category, DGWarning)]
        assert (len(got) == 3) == warn and (len(got) == 0) == (not warn), [str(r.message) for r in got]
        # outputs are valid either way
        assert abs(dt_g - dt_o) <= 1e-13 * dt_o and ch_g == ch_o and abs(k_g - k_o) <= 1e-13 * k_o
        assert st["n_ch_violation"] == (1 if warn else 0)
