"""hipGraph replay of the SSP-RK step (handles on a non-null stream) gives
bitwise the same states as direct launches, replay after replay, with eager
work and synchronisations between replays."""
import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("D,d,n,lim,field,rk", [(3, 2, 6, 0, "smooth", 3), (3, 3, 5, 7, "blast", 3),
                                                (2, 1, 32, 0, "smooth", 3), (3, 2, 6, 7, "blast", 5),
                                                (2, 2, 12, 0, "smooth", 2)])
def test_graph_replays_match_direct_launches(D, d, n, lim, field, rk):
    from paper_1806_02343_amd import DG
    print("case graph", D, d, n, lim, rk, flush=True)
    f = wl.Smooth(11, D) if field == "smooth" else wl.Blast(2000)
    s = torch.cuda.Stream()
    direct = DG(D, d, n, limiter=lim, rk_stages=rk)   # null stream: direct launches
    with torch.cuda.stream(s):
        graphed = DG(D, d, n, limiter=lim, stream=s.cuda_stream, rk_stages=rk)
        wa = graphed.empty_state()
        graphed.project_field(f, wa)
        if lim:
            graphed.limit(wa)
    s.synchronize()
    wb = direct.empty_state()
    direct.project_field(f, wb)
    if lim:
        direct.limit(wb)
    torch.cuda.synchronize()
    assert torch.equal(wa, wb)
    for rep in range(4):
        with torch.cuda.stream(s):
            graphed.step(wa, 1)
        direct.step(wb, 1)
        torch.cuda.synchronize()
        assert torch.equal(wa, wb), rep
        # eager work between replays
        wb.add_(0.0)
    # several steps per call reuse the same graph
    with torch.cuda.stream(s):
        graphed.step(wa, 3)
    direct.step(wb, 3)
    torch.cuda.synchronize()
    assert torch.equal(wa, wb)
