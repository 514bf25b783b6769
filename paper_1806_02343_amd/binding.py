"""ctypes binding of the C ABI in include/dg.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgmhd.so")

DG_OK, DG_EINVAL, DG_EUNSUPPORTED, DG_EHIP, DG_ENOMEM, DG_ENONFINITE, DG_ECH = 0, -1, -2, -3, -4, -5, -6
DG_GLM, DG_POWELL = 0, 1
DG_FP64, DG_FP32 = 0, 1
DG_LIM_TVB, DG_LIM_CHAR, DG_LIM_POS, DG_LIM_LEARNED = 1, 2, 4, 8
DG_MESH_UNIFORM, DG_MESH_OCTREE = 0, 1
DG_POWELL_Q_MEAN, DG_POWELL_Q_INTERP = 0, 1

EXPORTS = ["dg_init", "dg_layout", "dg_proj_points", "dg_project", "dg_nodal", "dg_amr_indicator", "dg_amr_plan",
           "dg_amr_leaves", "dg_amr_transfer", "dg_dt", "dg_rhs", "dg_rhs_noalloc", "dg_limit",
           "dg_step",
           "dg_mlp_scale", "dg_mlp_set", "dg_mlp_get", "dg_mlp_features", "dg_mlp_labels", "dg_mlp_record", "dg_mlp_forward",
           "dg_mlp_grad", "dg_mlp_train", "dg_time_kernel", "dg_autotune", "dg_last_error", "dg_destroy"]
MLP_NPARAM = 24833
AMR_FIELDS_RHO_B = (1 << 0) | (1 << 5) | (1 << 6) | (1 << 7)   # the paper's refinement fields


class dg_params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("degree", ctypes.c_int32), ("divb", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("rk_stages", ctypes.c_int32), ("limiter", ctypes.c_int32),
                ("powell_q", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("cfl_glm", ctypes.c_double),
                ("glm_cr", ctypes.c_double), ("glm_ch_fixed", ctypes.c_double),
                ("tvb_Mtilde", ctypes.c_double), ("tvb_beta", ctypes.c_double), ("tvb_eps", ctypes.c_double),
                ("eps_rho", ctypes.c_double), ("eps_p", ctypes.c_double), ("powell_eta", ctypes.c_double),
                ("mlp_lo", ctypes.c_double), ("mlp_hi", ctypes.c_double)]


class dg_mesh(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("box", ctypes.c_double * 3),
                ("nleaves", ctypes.c_int64), ("level", ctypes.POINTER(ctypes.c_int8)),
                ("ijk", ctypes.POINTER(ctypes.c_int32))]


class dg_limit_stats(ctypes.Structure):
    _fields_ = [("n_tvb_triggered", ctypes.c_int64), ("n_mlp_flagged", ctypes.c_int64),
                ("n_fallback", ctypes.c_int64), ("n_pos_scaled", ctypes.c_int64), ("n_floor", ctypes.c_int64),
                ("n_ch_violation", ctypes.c_int64),
                ("injected_mass", ctypes.c_double), ("injected_energy", ctypes.c_double),
                ("max_signal", ctypes.c_double), ("ch", ctypes.c_double)]


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dg error {code}: {msg}")
        self.code = code


class DGWarning(RuntimeWarning):
    """Warning-class status (DG_ECH): the call completed, its outputs are valid."""


_lib = None


def load_library(path=LIB_PATH):
    """Load libdgmhd.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdgmhd.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.dg_init.argtypes = [ctypes.POINTER(dg_params), ctypes.POINTER(dg_mesh), P, ctypes.POINTER(P)]
    lib.dg_layout.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)]
    lib.dg_proj_points.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I64)]
    lib.dg_project.argtypes = [P, P, I64, I64, P]
    lib.dg_nodal.argtypes = [P, P, I64, I64, P]
    lib.dg_amr_indicator.argtypes = [P, P, ctypes.c_uint32, P]
    lib.dg_amr_plan.argtypes = [P, P, ctypes.c_uint32, D, I32, ctypes.POINTER(I64)]
    lib.dg_amr_leaves.argtypes = [P, ctypes.POINTER(ctypes.c_int8), ctypes.POINTER(I32)]
    lib.dg_amr_transfer.argtypes = [P, P, P, P]
    lib.dg_dt.argtypes = [P, P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.dg_rhs.argtypes = [P, P, P, D, D]
    lib.dg_rhs_noalloc.argtypes = [P, P, P, D, D]
    lib.dg_limit.argtypes = [P, P, ctypes.POINTER(dg_limit_stats)]
    lib.dg_step.argtypes = [P, P, I32, ctypes.POINTER(D)]
    F32P = ctypes.POINTER(ctypes.c_float)
    lib.dg_mlp_scale.argtypes = [P, P, ctypes.POINTER(D)]
    lib.dg_mlp_set.argtypes = [P, F32P, ctypes.POINTER(D), ctypes.c_uint64]
    lib.dg_mlp_get.argtypes = [P, F32P]
    lib.dg_mlp_features.argtypes = [P, P, P]
    lib.dg_mlp_labels.argtypes = [P, P, P]
    lib.dg_mlp_record.argtypes = [P, P, P, P, I64, D, D, ctypes.c_uint64]
    lib.dg_mlp_forward.argtypes = [P, P, I64, P]
    lib.dg_mlp_grad.argtypes = [P, P, P, I64, F32P, F32P]
    lib.dg_mlp_train.argtypes = [P, P, P, I64, I32, I32, ctypes.c_float, ctypes.c_uint64, F32P]
    lib.dg_time_kernel.argtypes = [P, P, I32, I32, ctypes.POINTER(D)]
    lib.dg_autotune.argtypes = [P, P, ctypes.c_char_p, ctypes.POINTER(I32)]
    lib.dg_last_error.argtypes = [P]
    lib.dg_last_error.restype = ctypes.c_char_p
    lib.dg_destroy.argtypes = [P]
    lib.dg_destroy.restype = None
    for name in EXPORTS:
        if name not in ("dg_last_error", "dg_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class DG:
    """One handle of the library on the current HIP device.

    Arguments mirror dg_params / dg_mesh; state tensors are [nmodes][ld]
    torch tensors on the device (float64 or float32)."""

    def __init__(self, dim, degree, n, box=1.0, divb=DG_GLM, precision=DG_FP64, limiter=0, gamma=5.0 / 3.0,
                 cfl=0.3, cfl_glm=0.0, glm_cr=0.18, glm_ch_fixed=0.0, tvb_Mtilde=5.0, tvb_beta=2.0, tvb_eps=1e-8,
                 eps_rho=1e-12, eps_p=1e-12, powell_eta=0.2, mlp_lo=0.0, mlp_hi=0.0, stream=None, octree=None,
                 rk_stages=3, powell_q=0):
        """octree: optional (level[int8, C], ijk[int32, C x 3]) leaves on the level
        grids of the base grid n (kind DG_MESH_OCTREE)."""
        import torch
        self.torch = torch
        self.lib = load_library()
        self.dim, self.degree, self.divb, self.precision = dim, degree, divb, precision
        # the settings a regridded handle inherits
        self._kwargs = dict(divb=divb, precision=precision, limiter=limiter, gamma=gamma, cfl=cfl, cfl_glm=cfl_glm,
                            glm_cr=glm_cr, glm_ch_fixed=glm_ch_fixed, tvb_Mtilde=tvb_Mtilde, tvb_beta=tvb_beta,
                            tvb_eps=tvb_eps, eps_rho=eps_rho, eps_p=eps_p, powell_eta=powell_eta, mlp_lo=mlp_lo,
                            mlp_hi=mlp_hi, stream=stream, rk_stages=rk_stages, powell_q=powell_q)
        p = dg_params(dim, degree, divb, precision, rk_stages, limiter, powell_q, gamma, cfl, cfl_glm, glm_cr,
                      glm_ch_fixed,
                      tvb_Mtilde, tvb_beta, tvb_eps, eps_rho, eps_p, powell_eta, mlp_lo, mlp_hi)
        nn = list(n) if hasattr(n, "__len__") else [n] * dim
        bb = list(box) if hasattr(box, "__len__") else [box] * dim
        nn += [1] * (3 - len(nn))
        bb += [1.0] * (3 - len(bb))
        if octree is None:
            m = dg_mesh(DG_MESH_UNIFORM, (ctypes.c_int32 * 3)(*nn), (ctypes.c_double * 3)(*bb), 0, None, None)
            self.level = self.ijk = None
        else:
            import numpy as np
            self.level = np.ascontiguousarray(octree[0], dtype=np.int8)
            self.ijk = np.ascontiguousarray(octree[1], dtype=np.int32).reshape(-1, 3)
            m = dg_mesh(DG_MESH_OCTREE, (ctypes.c_int32 * 3)(*nn), (ctypes.c_double * 3)(*bb), len(self.level),
                        self.level.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                        self.ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self.n, self.box = nn[:dim], bb[:dim]
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        self._kwargs["stream"] = stream
        h = ctypes.c_void_p()
        rc = self.lib.dg_init(ctypes.byref(p), ctypes.byref(m), ctypes.c_void_p(stream), ctypes.byref(h))
        if rc != DG_OK:
            raise DGError(rc, self.lib.dg_last_error(None).decode())
        self.h = h
        nm, nc, ld = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.dg_layout(h, ctypes.byref(nm), ctypes.byref(nc), ctypes.byref(ld)))
        self.nmodes, self.ncells, self.ld = nm.value, nc.value, ld.value
        self.dtype = torch.float64 if precision == DG_FP64 else torch.float32

    def _check(self, rc):
        if rc == DG_ECH:
            import warnings
            warnings.warn(DGWarning(self.lib.dg_last_error(self.h).decode()), stacklevel=3)
        elif rc != DG_OK:
            raise DGError(rc, self.lib.dg_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def empty_state(self):
        return self.torch.zeros((self.nmodes, self.ld), dtype=self.dtype, device="cuda")

    def proj_points(self):
        import numpy as np
        npts = ctypes.c_int64()
        self._check(self.lib.dg_proj_points(self.h, None, ctypes.byref(npts)))
        xi = np.zeros(npts.value * self.dim)
        self._check(self.lib.dg_proj_points(self.h, xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            ctypes.byref(npts)))
        return xi.reshape(npts.value, self.dim)

    def project(self, prim, cell0, ncell, w):
        """prim: device float64 tensor [9][ncell][npts] of primitive values."""
        assert prim.dtype == self.torch.float64 and prim.is_contiguous()
        self._check(self.lib.dg_project(self.h, _ptr(prim), cell0, ncell, _ptr(w)))

    def nodal(self, w, cell0=0, ncell=None, out=None):
        """Conserved state at the projection points: device float64 tensor
        [nvar][npts][ncell] (nvar 9 for GLM, 8 for Powell)."""
        torch = self.torch
        ncell = self.ncells - cell0 if ncell is None else ncell
        nvar = 9 if self.divb == DG_GLM else 8
        npts = self.proj_points().shape[0]
        if out is None:
            out = torch.empty((nvar, npts, ncell), dtype=torch.float64, device="cuda")
        assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= nvar * npts * ncell
        self._check(self.lib.dg_nodal(self.h, _ptr(w), cell0, ncell, _ptr(out)))
        return out

    # ---------------------------------------------------------------- dynamic refinement
    def amr_indicator(self, w, fields=AMR_FIELDS_RHO_B):
        S = self.torch.empty(self.ncells, dtype=self.torch.float64, device="cuda")
        self._check(self.lib.dg_amr_indicator(self.h, _ptr(w), fields, _ptr(S)))
        return S

    def regrid(self, w, s_tilde=0.03, max_level=8, fields=AMR_FIELDS_RHO_B, **overrides):
        """One regrid (dg_amr_plan, dg_amr_leaves, a new handle on the planned
        leaves with this handle's settings updated by `overrides` (an octree
        handle needs glm_ch_fixed), dg_amr_transfer).  Returns the new handle
        and its state."""
        import numpy as np
        n = ctypes.c_int64()
        self._check(self.lib.dg_amr_plan(self.h, _ptr(w), fields, s_tilde, max_level, ctypes.byref(n)))
        level = np.zeros(n.value, dtype=np.int8)
        ijk = np.zeros((n.value, 3), dtype=np.int32)
        self._check(self.lib.dg_amr_leaves(self.h, level.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                                           ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        new = DG(self.dim, self.degree, tuple(self.n), box=tuple(self.box), octree=(level, ijk),
                 **{**self._kwargs, **overrides})
        w_new = new.empty_state()
        self._check(self.lib.dg_amr_transfer(self.h, _ptr(w), new.h, _ptr(w_new)))
        return new, w_new

    def dt(self, w):
        dt, ch, k = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.dg_dt(self.h, _ptr(w), ctypes.byref(dt), ctypes.byref(ch), ctypes.byref(k)))
        return dt.value, ch.value, k.value

    def rhs(self, w, dwdt, ch, kappa):
        self._check(self.lib.dg_rhs(self.h, _ptr(w), _ptr(dwdt), ch, kappa))

    def rhs_noalloc(self, w, dwdt, ch, kappa):
        self._check(self.lib.dg_rhs_noalloc(self.h, _ptr(w), _ptr(dwdt), ch, kappa))

    def limit(self, w, stats=False):
        if stats:
            s = dg_limit_stats()
            self._check(self.lib.dg_limit(self.h, _ptr(w), ctypes.byref(s)))
            return {k: getattr(s, k) for k, _ in dg_limit_stats._fields_}
        self._check(self.lib.dg_limit(self.h, _ptr(w), None))
        return None

    def step(self, w, nsteps=1, t=0.0):
        tt = ctypes.c_double(t)
        self._check(self.lib.dg_step(self.h, _ptr(w), nsteps, ctypes.byref(tt)))
        return tt.value

    def time_kernel(self, w, which, reps=10):
        """Mean ms per launch of one kernel of the step (0 face, 1 cell, 2 dt, 3 limiter)."""
        ms = ctypes.c_double()
        self._check(self.lib.dg_time_kernel(self.h, _ptr(w), which, reps, ctypes.byref(ms)))
        return ms.value

    def autotune(self, w, variant=-1, cache_path=None):
        """Pick (variant < 0) or force the cell-kernel tile variant; returns it."""
        v = ctypes.c_int32(variant)
        cp = cache_path.encode() if cache_path else None
        self._check(self.lib.dg_autotune(self.h, _ptr(w), cp, ctypes.byref(v)))
        return v.value

    # ---------------------------------------------------------------- learned indicator
    def mlp_scale(self, w):
        import numpy as np
        out = np.zeros(9)
        self._check(self.lib.dg_mlp_scale(self.h, _ptr(w), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def mlp_set(self, params, sigma=None, seed=0):
        import numpy as np
        sgp = None
        if sigma is not None:
            sg = np.ascontiguousarray(sigma, dtype=np.float64)
            assert sg.shape == (9,)
            sgp = sg.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        pp = None
        if params is not None:
            pp = np.ascontiguousarray(params, dtype=np.float32)
            assert pp.shape == (MLP_NPARAM,)
            pp = pp.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._check(self.lib.dg_mlp_set(self.h, pp, sgp, seed))

    def mlp_get(self):
        import numpy as np
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(self.lib.dg_mlp_get(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def mlp_features(self, w, X):
        self._check(self.lib.dg_mlp_features(self.h, _ptr(w), _ptr(X)))

    def mlp_labels(self, w, y):
        self._check(self.lib.dg_mlp_labels(self.h, _ptr(w), _ptr(y)))

    def mlp_record(self, X=None, y=None, counter=None, q_pos=1.0, q_neg=0.0, seed=0):
        if X is None:
            self._check(self.lib.dg_mlp_record(self.h, None, None, None, 0, 0.0, 0.0, 0))
        else:
            self._check(self.lib.dg_mlp_record(self.h, _ptr(X), _ptr(y), _ptr(counter), X.shape[0], q_pos, q_neg,
                                               seed))

    def mlp_forward(self, X, nrows, prob):
        self._check(self.lib.dg_mlp_forward(self.h, _ptr(X), nrows, _ptr(prob)))

    def mlp_grad(self, X, y, nrows):
        import numpy as np
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        loss = ctypes.c_float()
        self._check(self.lib.dg_mlp_grad(self.h, _ptr(X), _ptr(y), nrows,
                                         g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)))
        return loss.value, g

    def mlp_train(self, X, y, nrows, batch=4096, epochs=4, lr=1e-3, seed=0):
        import numpy as np
        losses = np.zeros(epochs, dtype=np.float32)
        self._check(self.lib.dg_mlp_train(self.h, _ptr(X), _ptr(y), nrows, batch, epochs, lr, seed,
                                          losses.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return losses

    def step_async(self, w, nsteps=1):
        self._check(self.lib.dg_step(self.h, _ptr(w), nsteps, None))

    def cell_centers(self, c0, nc):
        """Centres and sizes of cells c0 .. c0+nc-1 (uniform: index i + n0 (j + n1 k);
        octree: the leaves given at construction)."""
        torch = self.torch
        if self.level is not None:
            lv = torch.as_tensor(self.level[c0:c0 + nc].astype("int64"), device="cuda")
            ijk = torch.as_tensor(self.ijk[c0:c0 + nc, :self.dim].astype("float64"), device="cuda")
            h = (self.box[0] / self.n[0]) / (2.0 ** lv.to(torch.float64))
            return (ijk + 0.5) * h[:, None], h[:, None, None]
        idx = torch.arange(c0, c0 + nc, device="cuda", dtype=torch.int64)
        h = self.box[0] / self.n[0]
        cols, stride = [], 1
        for a in range(self.dim):
            cols.append(((idx // stride) % self.n[a]).to(torch.float64) * h + 0.5 * h)
            stride *= self.n[a]
        return torch.stack(cols, dim=1), h

    def project_field(self, field, w, chunk=1 << 16):
        """Evaluate a pointwise primitive field (callable x[P, D] -> dict, see
        workloads) at the library's projection points and project it into w.
        The point values are computed on the handle's stream, so that the
        library's kernels read them in order and their memory is not reused
        while a projection still reads it."""
        torch = self.torch
        if torch.cuda.current_stream().cuda_stream == self.stream:
            return self._project_field(field, w, chunk)
        with torch.cuda.stream(torch.cuda.ExternalStream(self.stream)):
            return self._project_field(field, w, chunk)

    def _project_field(self, field, w, chunk):
        torch = self.torch
        xi = torch.as_tensor(self.proj_points(), dtype=torch.float64, device="cuda")
        npts = xi.shape[0]
        for c0 in range(0, self.ncells, chunk):
            nc = min(chunk, self.ncells - c0)
            ctr, h = self.cell_centers(c0, nc)
            x = (ctr[:, None, :] + 0.5 * h * xi[None, :, :]).reshape(-1, self.dim)  # h: scalar or [nc,1,1]
            pr = field(x)
            comps = [pr["rho"], pr["v"][0], pr["v"][1], pr["v"][2], pr["p"], pr["B"][0], pr["B"][1], pr["B"][2],
                     pr["psi"]]
            comps = [c if isinstance(c, torch.Tensor) else torch.full_like(x[:, 0], float(c)) for c in comps]
            prim = torch.stack([c.to(torch.float64) for c in comps]).reshape(9, nc, npts).contiguous()
            self.project(prim, c0, nc, w)
            del prim, x
        return w
