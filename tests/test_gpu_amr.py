"""GPU parity on octree meshes with 2:1 hanging faces (GLM, fixed c_h):
right-hand side and SSP-RK3 steps against the oracle, and the peaks
workload's leaf generator driving both sides."""
import sys
import warnings

import numpy as np
import pytest

import workloads as wl
from oracle import dg
from oracle.amr import Octree
from parity_util import block_rel_max, rel_l1, to_cells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
G = 5.0 / 3.0


def small_tree(D, n0=4):
    t = Octree.uniform(D, n0)
    flags = np.array([all(1 <= c[a] <= 2 for a in range(D)) for _, c in t.leaves])
    t = t.refine(flags)
    flags = np.array([l == 1 and all(c[a] == 3 for a in range(D)) for l, c in t.leaves])
    return t.refine(flags).balanced().morton_sorted()


def pair(t, d, field, precision=0, ch=3.0):
    from paper_1806_02343_amd import DG
    D = t.D
    gpu = DG(D, d, t.n0, precision=precision, glm_ch_fixed=ch, octree=(t.levels(), t.coords()))
    wg = gpu.empty_state()
    gpu.project_field(field, wg)
    torch.cuda.synchronize()
    orc = dg.DG(t.mesh(), d, glm_ch_fixed=ch)
    wo = orc.project(dg.conserved_field(field, G, 9))
    return gpu, wg, orc, wo


@pytest.mark.parametrize("d", [1, 2, 3])
def test_amr_rhs_and_steps_match_oracle(d):
    print("case amr", d, flush=True)
    t = small_tree(3)
    gpu, wg, orc, wo = pair(t, d, wl.Smooth(77, 3))
    assert np.all(block_rel_max(to_cells(wg, orc.mesh.ncells), wo, orc) < 1e-13)
    r_o = orc.rhs(wo, 3.0, 1.5)
    out = gpu.empty_state()
    gpu.rhs(wg, out, 3.0, 1.5)
    torch.cuda.synchronize()
    assert np.all(block_rel_max(to_cells(out, orc.mesh.ncells), r_o, orc) < 1e-12)
    dto, _, _ = orc.timestep(wo)
    dtg, _, _ = gpu.dt(wg)
    assert abs(dtg - dto) <= 1e-13 * dto
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo)
    gpu.step(wg, 3)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=ch)
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("d", [1, 2, 3])
def test_amr_every_cell_variant_matches_oracle(d):
    """Every cell-kernel variant on an octree (LDS-tiled, matrix-core with the
    sub-face owner gather, persistent), with either face kernel (per face
    point, or matrix-core over tiles of one face class), gives the oracle's
    right-hand side."""
    print("case amr variants", d, flush=True)
    t = small_tree(3)
    gpu, wg, orc, wo = pair(t, d, wl.Smooth(79, 3))
    r_o = orc.rhs(wo, 3.0, 1.5)
    ran = 0
    for v in [c + 16 * f for f in range(4) for c in range(10)]:
        try:
            gpu.autotune(wg, variant=v)
        except Exception:
            continue
        out = gpu.empty_state()
        gpu.rhs(wg, out, 3.0, 1.5)
        torch.cuda.synchronize()
        err = block_rel_max(to_cells(out, orc.mesh.ncells), r_o, orc)
        assert np.all(err < 1e-12), (v, err)
        ran += 1
    assert ran >= 16


def test_amr_fp32_steps():
    print("case amr fp32", flush=True)
    t = small_tree(3)
    gpu, wg, orc, wo = pair(t, 2, wl.Smooth(78, 3), precision=1)
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo)
    gpu.step(wg, 3)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=ch)
    assert np.all(err < 1e-5), err


def test_peaks_leaves_small_mesh_matches_oracle():
    """The peaks workload's octree recipe on a 8^3 base grid (scaled radii)."""
    print("case peaks small", flush=True)
    pk = wl.Peaks(3000, npk=3, width=0.08)
    lv, ijk = wl.peaks_leaves(pk, n0=8, r1=0.25, r2=0.15)
    t = Octree.from_arrays(3, 8, lv, ijk)
    assert not t.balance_violations().any()
    # c_h above twice the largest signal speed sum_a(|v_a| + c)/D (about 3.2
    # here), so the runtime c_h check passes
    gpu, wg, orc, wo = pair(t, 2, pk, ch=3.5)
    for _ in range(2):
        wo, dt, ch, k = orc.step(wo)
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        gpu.step(wg, 2)
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=ch)
    assert np.all(err < 1e-12), err


def test_octree_rejects_unbalanced_or_incomplete_leaves():
    from paper_1806_02343_amd import DG, DGError
    t = small_tree(3)
    lv, ijk = t.levels(), t.coords()
    with pytest.raises(DGError):
        DG(3, 2, 4, glm_ch_fixed=3.0, octree=(lv[1:], ijk[1:]))   # a hole
    with pytest.raises(DGError):
        DG(3, 2, 4, glm_ch_fixed=0.0, octree=(lv, ijk))             # c_h not fixed
