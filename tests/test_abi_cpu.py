"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
symbol declared in include/dg.h, and rejects invalid arguments before any
device work."""
import ctypes
import os
import re

import pytest

from paper_1806_02343_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = B.load_library()
    names = declared_symbols()
    assert set(B.EXPORTS) == set(names)
    for n in names:
        assert hasattr(lib, n), n


def _params(**kw):
    p = dict(dim=3, degree=2, divb=B.DG_GLM, precision=B.DG_FP64, rk_stages=3, limiter=0, powell_q=0,
             gamma=5 / 3, cfl=0.3,
             cfl_glm=0.0, glm_cr=0.18, glm_ch_fixed=0.0, tvb_Mtilde=5.0, tvb_beta=2.0, tvb_eps=1e-8,
             eps_rho=1e-12, eps_p=1e-12, powell_eta=0.2, mlp_lo=0.0, mlp_hi=0.0)
    p.update(kw)
    return B.dg_params(**p)


def _mesh(n=(4, 4, 4), box=(1.0, 1.0, 1.0), kind=B.DG_MESH_UNIFORM):
    return B.dg_mesh(kind, (ctypes.c_int32 * 3)(*n), (ctypes.c_double * 3)(*box), 0, None, None)


@pytest.mark.parametrize("kw,mesh,code", [
    (dict(dim=4), {}, B.DG_EINVAL),
    (dict(degree=4), {}, B.DG_EUNSUPPORTED),
    (dict(degree=0), {}, B.DG_EUNSUPPORTED),
    (dict(divb=7), {}, B.DG_EINVAL),
    (dict(precision=3), {}, B.DG_EINVAL),
    (dict(rk_stages=4), {}, B.DG_EUNSUPPORTED),
    (dict(rk_stages=0), {}, B.DG_EUNSUPPORTED),
    (dict(rk_stages=6), {}, B.DG_EUNSUPPORTED),
    (dict(cfl=1.5), {}, B.DG_EINVAL),
    (dict(gamma=1.0), {}, B.DG_EINVAL),
    (dict(dim=4), {}, B.DG_EINVAL),
    (dict(powell_q=2, divb=B.DG_POWELL), {}, B.DG_EINVAL),
    (dict(powell_q=1), {}, B.DG_EINVAL),
    ({}, dict(n=(4, 0, 4)), B.DG_EINVAL),
    ({}, dict(box=(1.0, 2.0, 1.0)), B.DG_EINVAL),
])
def test_init_rejects_invalid_arguments_before_device_work(kw, mesh, code):
    lib = B.load_library()
    h = ctypes.c_void_p()
    rc = lib.dg_init(ctypes.byref(_params(**kw)), ctypes.byref(_mesh(**mesh)), None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert lib.dg_last_error(None)


def test_null_handle_calls_return_einval():
    lib = B.load_library()
    assert lib.dg_layout(None, None, None, None) == B.DG_EINVAL
    assert lib.dg_rhs(None, None, None, 1.0, 0.0) == B.DG_EINVAL
    assert lib.dg_rhs_noalloc(None, None, None, 1.0, 0.0) == B.DG_EINVAL
    assert lib.dg_step(None, None, 1, None) == B.DG_EINVAL
    lib.dg_destroy(None)


def test_struct_layouts_match_header():
    # field order and sizes of the ABI structs (6 int32 + 13 double, etc.)
    assert ctypes.sizeof(B.dg_params) == 7 * 4 + 4 + 13 * 8   # 7 int32, padding to the doubles
    assert ctypes.sizeof(B.dg_limit_stats) == 6 * 8 + 4 * 8
    assert ctypes.sizeof(B.dg_mesh) == 4 + 12 + 24 + 8 + 8 + 8
