"""dg_rhs_noalloc (workspace in the library's per-device scratch array, no
allocation) against dg_rhs on the same handle and state: bitwise equal, on
two calls in a row, the second on a smaller mesh (the array keeps the first
call's contents), for GLM and Powell, FP64 and FP32; meshes whose workspace
exceeds the array are refused before any device work."""
import sys

import numpy as np
import pytest

from oracle import dg
from parity_util import make_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _announce(*a):
    print("case", *a, flush=True)
    sys.stdout.flush()


def _rhs_both(gpu, wg, ch, kappa):
    ref = gpu.empty_state()
    gpu.rhs(wg, ref, ch, kappa)
    out = torch.full_like(ref, float("nan"))
    gpu.rhs_noalloc(wg, out, ch, kappa)
    torch.cuda.synchronize()
    return ref, out


@pytest.mark.parametrize("cases", [
    [(3, 3, 12, dg.GLM, 0), (3, 2, 5, dg.GLM, 0)],
    [(3, 2, 10, dg.POWELL, 0), (3, 1, 4, dg.POWELL, 0)],
    [(2, 1, 64, dg.GLM, 1), (2, 2, 9, dg.GLM, 1)],
], ids=["glm_fp64", "powell_fp64", "glm2d_fp32"])
def test_rhs_noalloc_matches_rhs_on_two_calls(cases):
    for (D, d, n, divb, prec) in cases:
        _announce("noalloc", D, d, n, divb, prec)
        gpu, wg, orc, wo = make_pair(D, d, n, divb, precision=prec)
        dt, ch, kappa = gpu.dt(wg)
        ch = ch if divb == dg.GLM else 0.0
        ref, out = _rhs_both(gpu, wg, ch, kappa)
        C = orc.mesh.ncells
        assert torch.equal(ref[:, :C], out[:, :C])
        # neither entry point writes the padding columns past the last cell
        assert bool(out[:, C:].isnan().all())
        # and against the oracle at the usual bound (FP64)
        if prec == 0:
            r_o = orc.rhs(wo, ch, kappa)
            r_g = out[:, :orc.mesh.ncells].double().cpu().numpy().T
            scale = np.abs(r_o).max()
            assert np.abs(r_g - r_o).max() <= 1e-11 * scale


def test_rhs_noalloc_refuses_meshes_beyond_the_array():
    from paper_1806_02343_amd.binding import DG_EINVAL, DGError
    from paper_1806_02343_amd import DG
    _announce("noalloc too large")
    gpu = DG(3, 3, 24)  # 13,824 cells x 3,456 B of face buffer > 32 MiB
    w = gpu.empty_state()
    out = torch.full_like(w, 7.0)
    with pytest.raises(DGError) as e:
        gpu.rhs_noalloc(w, out, 1.0, 0.0)
    assert e.value.code == DG_EINVAL
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
