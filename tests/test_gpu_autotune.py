"""The autotuner's schedule cache (dg_autotune with a cache path): keyed by
precision, dimension, degree, scheme, Powell q, cell count and, on octrees,
the level mix and the number of faces; a second handle of the same
configuration takes the cached schedule."""
import json
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.amr import Octree

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _tree(flag_cells):
    t = Octree.uniform(3, 4)
    t = t.refine(np.array([c in flag_cells for _, c in t.leaves])).balanced().morton_sorted()
    return t


def test_schedule_cache_keys_and_reuse(tmp_path):
    from paper_1806_02343_amd import DG
    print("case autotune cache", flush=True)
    sys.stdout.flush()
    path = str(tmp_path / "sched.json")
    g = DG(3, 2, 6)
    w = g.empty_state()
    g.project_field(wl.Smooth(5, 3), w)
    v1 = g.autotune(w, cache_path=path)
    g2 = DG(3, 2, 6)
    w2 = g2.empty_state()
    g2.project_field(wl.Smooth(5, 3), w2)
    assert g2.autotune(w2, cache_path=path) == v1
    # octrees: the key carries the leaves per level and the number of faces
    ta = _tree({(1, 1, 1)})
    tb = _tree({(1, 1, 1), (3, 3, 3)})
    keys = []
    for t in (ta, tb):
        h = DG(3, 2, 4, glm_ch_fixed=3.0, octree=(t.levels(), t.coords()))
        wh = h.empty_state()
        h.project_field(wl.Smooth(5, 3), wh)
        h.autotune(wh, cache_path=path)
    with open(path) as fh:
        text = fh.read()
    keys = [ln.split('"')[1] for ln in text.splitlines() if '"' in ln]
    octree_keys = [k for k in keys if "/L" in k]
    assert len(octree_keys) == 2, keys
    assert any("/L0:63,1:8,/F" in k for k in octree_keys) and any("/L0:62,1:16,/F" in k for k in octree_keys), keys
    assert any(k.startswith("sched/p0/D3/d2/b0/q0/C216") and "/L" not in k for k in keys)
