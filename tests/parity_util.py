"""Shared helpers of the GPU parity tests: build an oracle scheme and a HIP
handle for the same configuration and seeded input, and compare them."""
import numpy as np

import workloads as wl
from oracle import dg
from oracle.quadrature import tensor_rule

G = 5.0 / 3.0


def make_pair(D, d, n, divb=0, precision=0, box=1.0, field=None, limiter=0, cfl=0.3, **kw):
    import torch
    from paper_1806_02343_amd import DG
    field = field if field is not None else wl.Smooth(1000 * D + d, D)
    gpu = DG(D, d, n, box=box, divb=divb, precision=precision, limiter=limiter, cfl=cfl, **kw)
    wg = gpu.empty_state()
    gpu.project_field(field, wg)
    torch.cuda.synchronize()
    orc = dg.DG(dg.Mesh.uniform(D, n, box), d, divb=divb, cfl=cfl)
    wo = orc.project(dg.conserved_field(field, G, orc.nvar))
    return gpu, wg, orc, wo


def to_cells(t, ncells):
    """[nmodes][ld] device tensor -> oracle layout [cell][mode] (float64 numpy)."""
    return t[:, :ncells].double().cpu().numpy().T.copy()


def rel_l1(orc, w_test, w_ref, ch=1.0):
    """Per-variable relative L1 error of nodal values at (d+3)^D points
    (eq. lp_norm); psi is measured against c_h ||B||_1."""
    xq, wq = tensor_rule(orc.d + 3, orc.D)
    tabs = orc._basis_at(xq)
    Ut = orc.nodal(w_test, tabs=tabs)
    Ur = orc.nodal(w_ref, tabs=tabs)
    err = (np.abs(Ut - Ur) * wq).sum(axis=(1, 2))
    ref = (np.abs(Ur) * wq).sum(axis=(1, 2))
    out = err / np.maximum(ref, 1e-300)
    if orc.nvar == 9:
        bn = ref[5:8].sum()
        out[8] = err[8] / max(ch * bn, 1e-300)
    return out


def block_rel_max(a, b, orc, floor=1e-3):
    """max |a-b| / max |b| per variable block (modal arrays [cell][mode]).
    The denominator is floored at `floor` x the largest block maximum, so a
    block that is zero in exact arithmetic (e.g. momentum of a state at rest)
    is judged against the state's scale instead of its own rounding noise."""
    res = []
    n = orc.n
    gmax = max(np.abs(b).max(), 1e-300)
    for j in range(len(orc.leg_vars)):
        sl = slice(j * n, (j + 1) * n)
        res.append(np.abs(a[:, sl] - b[:, sl]).max() / max(np.abs(b[:, sl]).max(), floor * gmax))
    if orc.nldf:
        sl = slice(len(orc.leg_vars) * n, None)
        res.append(np.abs(a[:, sl] - b[:, sl]).max() / max(np.abs(b[:, sl]).max(), floor * gmax))
    return np.array(res)
