"""Throughput benchmark of the DG MHD hot path on one MI355X.

One step = one SSP-RK3 time step of the whole path (time-step reduction,
then per stage the face-flux kernel, the cell kernel and the limiters) over
the full workload, inputs resident in HBM; the step replays one captured
hipGraph.  The metric is DoF-updates per second per RK stage:
N_DoF x 3 x steps / wall time.

Default workload (the metric's comparison): 3-D periodic 128^3, degree 3,
GLM, 8 seeded over-pressured spheres, characteristic TVB + positivity
limiters, CFL 0.3.  `value` is the FP64 plain method; the same JSON line
carries the FP32 path and the FP32 path with the learned troubled-cell
indicator (trained during untimed setup on other seeds), each with its
relative L1 distance to the FP64 state after the timed steps.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG DoF-updates/sec per RK stage, FP64 plain vs FP32+learned limiter at L1 tol"
PEAK_FP64 = 78.6e12   # MI355X FP64 (vector = matrix) flop/s
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12
L1_TOL = 1e-5

# default step counts of each workload (the number of steps it is specified with)
DEFAULT_STEPS = {"blast128": 50, "smooth64": 20, "smooth32_2d": 10, "peaks_amr": 30}
VARS = ["rho", "mx", "my", "mz", "E", "Bx", "By", "Bz"]

WORKLOADS = {
    # name: (D, d, n, divb, limiter, seed-config, description)
    "blast128": (3, 3, 128, 0, 7, 2, "3-D periodic 128^3, degree 3 (20 modes/var), GLM, 8 seeded over-pressured "
                                     "spheres, characteristic TVB + positivity limiters, SSP-RK3, CFL 0.3"),
    "smooth64": (3, 2, 64, 1, 0, 1, "3-D periodic 64^3, degree 2, Powell scheme with the LDF basis for B, smooth "
                                    "seeded IC (random Fourier modes, B = curl A), SSP-RK3, CFL 0.3"),
    "smooth32_2d": (2, 1, 32, 0, 0, 0, "2-D periodic 32^2, degree 1, GLM, smooth seeded IC, SSP-RK3, CFL 0.3"),
    "peaks_amr": (3, 2, 64, 0, 0, 3, "3-D octree: base 64^3, 2 levels around 16 seeded Gaussian density peaks "
                                     "(1,520,093 leaves), degree 2, GLM with fixed c_h, hanging faces, SSP-RK3, "
                                     "CFL 0.3"),
}


def cell_flops(D, d, divb, moments=False):
    """Algorithmic flops per cell of one cell-kernel launch (stage): the dense
    contractions of the weak form plus a fixed pointwise flux cost.  moments:
    the surface lift takes the face moments (polynomials of degree <= d in the
    face coordinates) instead of the face-point fluxes."""
    from oracle.basis import n_div, n_modes
    n = n_modes(D, d)
    P = d + 1
    Q, FP = P ** D, P ** (D - 1)
    if moments:
        FP = P if D == 2 else P * (P + 1) // 2
    nleg = 9 if divb == 0 else (5 if D == 3 else 6)
    nldf = 0 if divb == 0 else n_div(D, d)
    nodal = 2 * Q * (nleg * n + D * nldf)                  # modal -> nodal at volume points
    flux = Q * D * 45                                     # analytic flux per point and axis
    vol = 2 * Q * D * (nleg * n + D * nldf)               # volume projection
    surf = 2 * D * 2 * FP * (nleg * n + D * nldf)         # surface lift of 2D faces
    powell = surf if divb == 1 else 0
    update = 6 * (nleg * n + nldf)
    return nodal + flux + vol + surf + powell + update


def rel_l1_nodal(ga, wa, gb, wb, nvar_cmp=8, chunk=1 << 15):
    """Relative L1 distance of two states per conserved variable (eq. lp_norm
    with the (d+3)^D Gauss rule of the projection points): sum_K sum_p w_p
    |a - b| / sum_K sum_p w_p |b| for rho, m, E, B; returns (max, list)."""
    import numpy as np
    import torch
    x1, w1 = np.polynomial.legendre.leggauss(ga.degree + 3)
    xi = ga.proj_points()
    idx = np.abs(xi[:, :, None] - x1[None, None, :]).argmin(axis=-1)
    wq = torch.as_tensor(np.prod(w1[idx], axis=1), device="cuda")[None, :, None]
    err = torch.zeros(nvar_cmp, dtype=torch.float64, device="cuda")
    ref = torch.zeros_like(err)
    for c0 in range(0, ga.ncells, chunk):
        nc = min(chunk, ga.ncells - c0)
        # the handles may write on streams of their own: the previous chunk's
        # reductions must be done before the buffers are rewritten, and the
        # values must be written before they are read
        torch.cuda.synchronize()
        A = ga.nodal(wa, c0, nc)[:nvar_cmp]
        B = gb.nodal(wb, c0, nc)[:nvar_cmp]
        torch.cuda.synchronize()
        _, h = ga.cell_centers(c0, nc)        # octree cells carry their own size
        vol = h.reshape(1, 1, -1) ** ga.dim if isinstance(h, torch.Tensor) else 1.0
        err += ((A - B).abs() * wq * vol).sum(dim=(1, 2))
        ref += (B.abs() * wq * vol).sum(dim=(1, 2))
        del A, B
    per = (err / ref).tolist()
    return max(per), per


def timed_run(gpu, w0, steps, warmup):
    import torch
    w = w0.clone()
    gpu.step(w, warmup)
    w.copy_(w0)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    gpu.step_async(w, steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), w


def make_handle(D, d, n, divb, limiter, prec, stream, octree=None, ch=0.0, lo=0.0):
    from paper_1806_02343_amd import DG
    return DG(D, d, n, divb=divb, precision=prec, limiter=limiter, cfl=0.3, stream=stream, octree=octree,
              glm_ch_fixed=ch, mlp_lo=lo, mlp_hi=0.5)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's own count)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="blast128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with one device copy of 1 GiB (the calibration kernel of the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the design notes describe how the path would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wl
    from paper_1806_02343_amd import DG_LIM_LEARNED

    D, d, n, divb, limiter, cfg, desc = WORKLOADS[args.workload]
    if args.steps is None:
        args.steps = DEFAULT_STEPS[args.workload]
    stream = torch.cuda.Stream()          # non-null stream: each step replays one captured hipGraph
    torch.cuda.set_stream(stream)
    octree, ch = None, 0.0
    if args.workload == "peaks_amr":
        pk = wl.Peaks(3000)
        octree = wl.peaks_leaves(pk)
        # c_h fixed at twice the largest signal speed sum_a(|v_a| + c)/D of the
        # initial state (background density 1 has the largest sound and Alfven speeds)
        B2 = sum(b * b for b in pk.B0)
        c = np.sqrt((5.0 / 3.0 * 1.0 + B2) / 1.0)
        ch = 2.0 * (sum(abs(v) for v in pk.V0) + 3 * c) / 3
        field = pk
    else:
        field = wl.config_field(cfg)

    runs = {}

    def run(tag, prec, lim, extra=None, lo=0.0):
        gpu = make_handle(D, d, n, divb, lim, prec, stream.cuda_stream, octree, ch, lo)
        w0 = gpu.empty_state()
        gpu.project_field(field, w0)
        if extra:
            extra(gpu, w0)
        if lim:
            gpu.limit(w0)
        variant = gpu.autotune(w0)
        ms, w = timed_run(gpu, w0, args.steps, args.warmup)
        ndof = gpu.nmodes * gpu.ncells
        r = dict(ms=ms, ndof=ndof, value=ndof * 3 * args.steps / (ms / 1e3), w=w, gpu=gpu, variant=variant,
                 k_face=gpu.time_kernel(w0, 0, 5), k_cell=gpu.time_kernel(w0, 1, 6), k_dt=gpu.time_kernel(w0, 2, 5),
                 k_limit=gpu.time_kernel(w0, 3, 5) if lim else 0.0)
        print(f"# {tag}: ms/step={ms / args.steps:.3f} face={r['k_face']:.3f} cell={r['k_cell']:.3f} "
              f"dt={r['k_dt']:.3f} limit={r['k_limit']:.3f} (ms/launch) variant={variant}", file=sys.stderr,
              flush=True)
        runs[tag] = r
        return r

    r64 = run("fp64", 0, limiter)
    if not args.no_fp32:
        run("fp32", 1, limiter)
    learned_info = None
    if limiter and not args.no_learned and not args.no_fp32 and args.workload == "blast128":
        from paper_1806_02343_amd.learned import false_negative_rate, train_indicator
        t0 = time.perf_counter()
        info = train_indicator(wl, n=n, d=d, stream=stream.cuda_stream)
        t_train = time.perf_counter() - t0
        print(f"# trained indicator: rows={info['n_train']} pos_frac={info['pos_frac_train']:.3f} "
              f"losses={info['losses']} lo={info['lo']:.4f} val_fn={info['val_fn_rate']:.4f} "
              f"({t_train:.1f}s)", file=sys.stderr, flush=True)

        def install(gpu, w0):
            gpu.mlp_set(info["params"], info["sigma"])

        rl = run("fp32_learned", 1, limiter | DG_LIM_LEARNED, install, info["lo"])
        # the gate on the evaluated workload itself, from the state the timed
        # steps ended in: the share of cells whose plain detector it skips, and
        # over two more recorded steps the positives of the plain detector that
        # it would have skipped
        g = rl["gpu"]
        w = rl["w"].clone()
        st = g.limit(w.clone(), stats=True)
        gate_skip = 1.0 - (st["n_fallback"] + st["n_mlp_flagged"]) / g.ncells
        cap = 1 << 21
        X = torch.zeros((cap, 256), dtype=torch.int16, device="cuda")
        y = torch.zeros(cap, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        g.mlp_record(X, y, cnt, q_pos=1.0, q_neg=0.02, seed=99)
        g.step(w, 2)
        g.mlp_record(None)
        torch.cuda.synchronize()
        nrec = min(int(cnt.item()), cap)
        fn, skip, _, _ = false_negative_rate(g, X, y, nrec, info["lo"])
        learned_info = dict(train_rows=info["n_train"], train_seeds=info["n_train_seeds"],
                            train_pos_frac=info["pos_frac_train"], val_skip_frac=info["val_skip_frac"],
                            losses=info["losses"], gate_lo=info["lo"], val_fn_rate=info["val_fn_rate"],
                            eval_fn_rate=fn, gate_skip_frac=gate_skip, train_seconds=t_train)

    ncells = r64["gpu"].ncells
    cv = r64["variant"] & 15
    mfma = cv >= 4
    # the matrix-core cell kernels lift face moments (GLM on uniform and
    # octree grids, 3-D Powell with the cell-mean q-dagger); 2-D Powell lifts
    # point values
    flops_launch = cell_flops(D, d, divb, moments=mfma and (divb == 0 or D == 3)) * ncells
    achieved = flops_launch / (r64["k_cell"] / 1e3)
    if divb:
        kname = ("k_cell_mfma_powell_p" if cv == 6 else "k_cell_mfma_powell") if mfma else "k_cell"
    else:
        kname = ("k_cell_mfma_p" if cv >= 8 else "k_cell_mfma") if mfma else "k_cell"
    roof = {"kernel": kname, "bound": "mfma" if mfma else "alu",
            "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
            "traffic": measured_traffic(args.workload, r64["variant"]) if mfma else None,
            "ms_per_launch": r64["k_cell"], "flops_per_launch": flops_launch}
    line = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "dim": D, "degree": d, "cells": ncells,
                   "n_dof": r64["ndof"], "divb": "powell+ldf" if divb else "glm", "limiter": limiter},
        "roofline": roof,
    }
    for tag in ("fp32", "fp32_learned"):
        if tag in runs:
            r = runs[tag]
            ent = {"value": r["value"], "ms_per_step": r["ms"] / args.steps, "speedup_vs_fp64": r["value"] / r64["value"]}
            rel, per = rel_l1_nodal(r["gpu"], r["w"], r64["gpu"], r64["w"])
            ent["rel_l1_vs_fp64"] = rel
            ent["rel_l1_per_var"] = dict(zip(VARS, per))
            ent["within_l1_tol"] = rel <= L1_TOL
            line[tag] = ent
    if learned_info:
        line["fp32_learned"].update(learned_info)
    if not args.no_cpu and args.workload != "peaks_amr":
        line["cpu_baseline"] = cpu_baseline(D, d, divb, cfg, limiter)
    print(json.dumps(line), flush=True)
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()


KERNEL_SOURCES = ["dg_kernels.hip", "dg_kernels.h", "dg_physics.h", "dg_limiters.inc"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1806_02343_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, variant):
    """HBM bytes per launch of the FP64 cell kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the
    reading of a 1 GiB copy), or None when the summary is missing, has no
    entry for the cell variant in use, or was taken from other kernel
    sources."""
    path = os.path.join(ROOT, "profiles", f"k_cell_mfma_{workload}_fp64_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for ln in fh:
            if "=" in ln and not ln.lstrip().startswith("#"):
                k, v = ln.split("=", 1)
                kv[k.strip()] = v.strip()
    key = f"traffic_bytes_per_launch_cell_variant_{variant & 15}"
    if kv.get("source_sha256") != kernel_source_hash() or key not in kv:
        return None
    return float(kv[key])


def cpu_baseline(D, d, divb, cfg, limiter, nsteps=2):
    """The FP64 oracle timed on the host on a bounded sample of the workload:
    two SSP-RK3 steps of the same scheme (limiters included) on a 24^3 (3-D)
    or 64^2 (2-D) grid of the same initial-condition family."""
    from threadpoolctl import threadpool_info

    import workloads as wl
    from oracle import dg, limiters
    nsample = 24 if D == 3 else 64
    orc = dg.DG(dg.Mesh.uniform(D, nsample), d, divb=divb)
    w = orc.project(dg.conserved_field(wl.config_field(cfg), 5.0 / 3.0, orc.nvar))
    lim = limiters.make_stage_limiter(orc, limiter) if limiter else None
    if lim:
        w = lim(w)
    t0, c0 = time.perf_counter(), time.process_time()
    for _ in range(nsteps):
        w, dt, ch, k = orc.step(w, limiter=lim)
    sec, cpu = time.perf_counter() - t0, time.process_time() - c0
    ndof = orc.nmodes * orc.mesh.ncells
    blas = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    # cores: the average number of cores the process kept busy (CPU time over
    # wall time); NumPy's elementwise work runs on one core, only the BLAS
    # products use the thread pool
    return {"value": ndof * 3 * nsteps / sec, "unit": "DoF-updates/s", "cores": round(cpu / sec, 2), "kind": "oracle",
            "host_cpus": os.cpu_count(), "cpu_model": model, "blas_threads": blas,
            "sample": f"{nsteps} SSP-RK3 steps of the same scheme on {nsample}^{D} cells ({ndof} DoF), {sec:.2f} s "
                      f"wall, {cpu:.2f} s CPU; elementwise NumPy work on one core, BLAS products on "
                      f"{blas} threads"}


if __name__ == "__main__":
    main()
