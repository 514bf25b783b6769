"""Shock problems of the paper's test section on the GPU (Sec. 5.3: Orszag-Tang
vortex, rotor, 2-D and 3-D blast waves; Sec. 5.4: field-loop advection), with
the paper's default scheme (degree 2, Powell with LDF field or GLM cleaning,
characteristic TVB limiter with M~ = 5, positivity floors 1e-12, SSP-RK3).

* Parity: three limited steps of every problem against the oracle at a small
  size, FP64 to 1e-12.
* Robustness runs at 128^2 (48^3 for the 3-D blast) to the paper's final
  times.  The paper's figures carry no numbers to compare with, so these
  runs check what holds at any resolution: mass conserved to rounding; the
  total energy conserved to rounding under GLM and, under the Powell
  scheme, drifting by no more than the paper's 0.6 % for the Orszag-Tang
  vortex at 128^2 up to t = 1; positive cell-mean density and pressure; the
  point symmetry of the Orszag-Tang vortex; a bounded divergence norm
  (eq. divb-total); and the 3-D blast's contrast between the schemes (Powell
  keeps the background pressure, GLM needs the pressure floor).

Diagnostics are evaluated on the host by the oracle's own routines from the
GPU state."""
import math
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import dg, limiters
from parity_util import rel_l1, to_cells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _announce(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


# name -> (D, field factory(n), final time, gamma, box)
PROBLEMS = {
    "orszag_tang": (2, lambda n: wl.OrszagTang(), 1.0, 5.0 / 3.0, 1.0),
    "rotor": (2, lambda n: wl.Rotor(), 0.15, 1.4, 1.0),
    "blast2d": (2, lambda n: wl.Blast2D(), 0.2, 5.0 / 3.0, 1.0),
    "blast2d_b10": (2, lambda n: wl.Blast2D(B0=10.0), 0.2, 5.0 / 3.0, 1.0),
    "blast3d": (3, lambda n: wl.Blast3D(n), 0.01, 1.4, 1.0),
    "loop": (2, lambda n: wl.Loop(), 2.0, 5.0 / 3.0, 2.0),
}


def _pair(name, n, divb, d=2, limiter=7):
    from paper_1806_02343_amd import DG
    D, fac, tf, gamma, box = PROBLEMS[name]
    field = fac(n)
    gpu = DG(D, d, n, box=box, divb=divb, limiter=limiter, gamma=gamma)
    wg = gpu.empty_state()
    gpu.project_field(field, wg)
    torch.cuda.synchronize()
    orc = dg.DG(dg.Mesh.uniform(D, n, box), d, divb=divb, gamma=gamma)
    wo = orc.project(dg.conserved_field(field, gamma, orc.nvar))
    return gpu, wg, orc, wo, tf


@pytest.mark.parametrize("name,n,divb", [("orszag_tang", 16, dg.POWELL), ("rotor", 32, dg.POWELL),
                                         ("blast2d", 24, dg.POWELL), ("blast3d", 8, dg.POWELL),
                                         ("loop", 16, dg.POWELL), ("orszag_tang", 16, dg.GLM),
                                         ("blast3d", 8, dg.GLM)])
def test_shock_problem_steps_match_oracle(name, n, divb):
    _announce("shock parity", name, n, divb)
    gpu, wg, orc, wo, _ = _pair(name, n, divb)
    olim = limiters.make_stage_limiter(orc, 7)
    wo = olim(wo)
    gpu.limit(wg)
    t_o = 0.0
    for _ in range(3):
        wo, dt, ch, k = orc.step(wo, limiter=olim)
        t_o += dt
    t_g = gpu.step(wg, 3)
    assert abs(t_g - t_o) <= 1e-12 * t_o
    err = rel_l1(orc, to_cells(wg, orc.mesh.ncells), wo, ch=max(ch, 1.0))
    assert np.all(err < 1e-12), err


def _diagnostics(orc, wg):
    w = to_cells(wg, orc.mesh.ncells)
    Ub = orc.cell_means(w)
    vol = orc.mesh.h[0] ** orc.D
    g = orc.gamma
    p = (g - 1.0) * (Ub[4] - 0.5 * (Ub[1] ** 2 + Ub[2] ** 2 + Ub[3] ** 2) / Ub[0]
                     - 0.5 * (Ub[5] ** 2 + Ub[6] ** 2 + Ub[7] ** 2))
    out = dict(mass=Ub[0].sum() * vol, energy=Ub[4].sum() * vol, rho_min=Ub[0].min(), p_min=p.min(),
               emag=0.5 * (Ub[5] ** 2 + Ub[6] ** 2 + Ub[7] ** 2).sum() * vol, w=w)
    if orc.divb == dg.POWELL:
        # eq. divb-total; the LDF field has no volume divergence, so |div B|_K
        # is the face-jump term of eq. divb-cell
        out["divb1"] = orc.divb_face_jump(w).mean()
    return out


def _run(name, n, divb, marks=4):
    gpu, wg, orc, _, tf = _pair(name, n, divb)
    gpu.limit(wg)
    d0 = _diagnostics(orc, wg)
    hist, t = [], 0.0
    for k in range(marks):
        tm = tf * (k + 1) / marks
        while t < tm:
            t += gpu.step(wg, 20)
        hist.append((t, _diagnostics(orc, wg)))
        h = hist[-1][1]
        print(f"{name} divb={divb} t={t:.4f} dmass={h['mass'] / d0['mass'] - 1:.2e} "
              f"dE={h['energy'] / d0['energy'] - 1:.2e} emag={h['emag'] / d0['emag']:.4f} "
              f"rho_min={h['rho_min']:.3e} p_min={h['p_min']:.3e} divb1={h.get('divb1', float('nan')):.3e}",
              flush=True)
    return d0, hist, orc


@pytest.mark.parametrize("divb", [dg.POWELL, dg.GLM])
def test_orszag_tang_vortex(divb):
    n = int(os.environ.get("DG_OT_N", "128"))
    _announce("orszag-tang", n, divb)
    d0, hist, orc = _run("orszag_tang", n, divb)
    for t, h in hist:
        assert abs(h["mass"] / d0["mass"] - 1.0) < 1e-11
        assert h["rho_min"] > 0.01 and h["p_min"] > 0.005
        dE = abs(h["energy"] / d0["energy"] - 1.0)
        if divb == dg.POWELL:
            # the paper: E_tot deviates by at most 0.6 % at 128^2 (0.3 % at 512^2) up to t = 1
            assert dE <= (0.006 if n <= 128 else 0.003), (t, dE)
            assert h["divb1"] < 3.0
        else:
            assert dE < 1e-11, (t, dE)
    # point symmetry about the box centre: rho(x) = rho(1 - x)
    r = hist[-1][1]["w"][:, 0].reshape(n, n)
    assert np.abs(r - r[::-1, ::-1]).max() < 1e-8 * np.abs(r).max()


@pytest.mark.parametrize("name", ["rotor", "blast2d", "blast2d_b10"])
@pytest.mark.parametrize("divb", [dg.POWELL, dg.GLM])
def test_2d_shock_problems_stay_positive_and_conservative(name, divb):
    """Rotor and 2-D blast (B0 = 1 and the strongly magnetised B0 = 10):
    mass to rounding, positive means, bounded energy drift.  GLM at B0 = 10
    behaves like the 3-D blast: cleaning waves in the low-beta background
    drive the pressure to the floor once, whose energy the tally reports."""
    _announce("2-D shock", name, divb)
    d0, hist, orc = _run(name, 128, divb)
    floor_expected = divb == dg.GLM and name == "blast2d_b10"
    for t, h in hist:
        assert abs(h["mass"] / d0["mass"] - 1.0) < 1e-11
        assert h["rho_min"] > 0.05, (t, h["rho_min"])
        # at the floor the host's mean pressure carries the rounding of E ~ 50
        assert h["p_min"] > (0.5e-12 if floor_expected else 1e-3), (t, h["p_min"])
        dE = abs(h["energy"] / d0["energy"] - 1.0)
        assert dE < (0.01 if divb == dg.POWELL else 1e-3 if floor_expected else 1e-11), (t, dE)


def test_blast3d_powell_keeps_pressure_glm_needs_the_floor():
    """The strongly magnetised 3-D blast (Sec. 5.3.7): under the Powell
    scheme the background keeps its pressure (no floor fires); under GLM the
    cleaning waves drive the background pressure to the floor, which the
    positivity limiter catches (the run still completes)."""
    _announce("blast3d")
    d0, hp, _ = _run("blast3d", 48, dg.POWELL, marks=2)
    for t, h in hp:
        assert abs(h["mass"] / d0["mass"] - 1.0) < 1e-11
        assert h["rho_min"] > 0.05 and h["p_min"] > 0.09, (t, h["p_min"])
        assert abs(h["energy"] / d0["energy"] - 1.0) < 2e-3
    d0g, hg, _ = _run("blast3d", 48, dg.GLM, marks=2)
    assert hg[-1][1]["p_min"] < 1e-6
    assert abs(hg[-1][1]["mass"] / d0g["mass"] - 1.0) < 1e-11


@pytest.mark.parametrize("divb", [dg.POWELL, dg.GLM])
def test_field_loop_advection(divb):
    """One period of the field loop (t = 2 on [-1,1]^2 with v = (2, 1)):
    the magnetic energy decays by less than 3 %, the total energy is
    conserved to within 1e-8 (the Powell terms do work only through the
    small divergence), and the divergence norm (eq. divb-total) stays below
    a fifth of the loop's field strength per unit length."""
    _announce("loop", divb)
    d0, hist, orc = _run("loop", 128, divb)
    for t, h in hist:
        assert abs(h["mass"] / d0["mass"] - 1.0) < 1e-11
        assert 0.97 < h["emag"] / d0["emag"] <= 1.0
        assert abs(h["energy"] / d0["energy"] - 1.0) < (1e-8 if divb == dg.POWELL else 1e-11)
        if divb == dg.POWELL:
            assert h["divb1"] < 0.2 * wl.Loop.A0
