"""Throughput benchmark of the DG MHD hot path on one MI355X.

One step = one SSP-RK3 time step of the whole path (time-step reduction, and
per stage the face-flux kernel, the cell kernel and the limiters) over the
full workload, inputs resident in HBM.  The metric is DoF-updates per second
per RK stage: N_DoF x 3 x steps / wall time.

Prints one JSON line (see the repository's design notes for every field).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG DoF-updates/sec per RK stage, FP64 plain vs FP32+learned limiter at L1 tol"
PEAK_FP64 = 78.6e12   # MI355X FP64 vector = matrix peak (flop/s)
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12

WORKLOADS = {
    # name: (D, d, n, divb, limiter, seed-config, description)
    "cfg1": (3, 2, 64, 1, 0, 1, "3-D periodic 64^3, degree 2, Powell scheme with the LDF basis for B, "
                                 "smooth seeded IC (random Fourier modes, B = curl A), SSP-RK3, CFL 0.3"),
    "cfg0": (2, 1, 32, 0, 0, 0, "2-D periodic 32^2, degree 1, GLM, smooth seeded IC, SSP-RK3, CFL 0.3"),
    "cfg2": (3, 3, 128, 0, 7, 2, "3-D periodic 128^3, degree 3, GLM, 8 seeded over-pressured spheres, "
                                  "characteristic TVB + positivity limiters, SSP-RK3, CFL 0.3"),
}


def cell_flops(D, d, divb):
    """Algorithmic flops per cell of one cell-kernel launch (stage): the dense
    contractions of the weak form plus a fixed pointwise flux cost."""
    from oracle.basis import n_div, n_modes
    n = n_modes(D, d)
    P = d + 1
    Q, FP = P ** D, P ** (D - 1)
    nleg = 9 if divb == 0 else (5 if D == 3 else 6)
    nldf = 0 if divb == 0 else n_div(D, d)
    nodal = 2 * Q * (nleg * n + D * nldf)                  # modal -> nodal at volume points
    flux = Q * D * 45                                     # analytic flux per point and axis
    vol = 2 * Q * D * (nleg * n + D * nldf)               # volume projection
    surf = 2 * D * 2 * FP * (nleg * n + D * nldf)         # surface lift of 2D faces
    powell = surf if divb == 1 else 0
    update = 6 * (nleg * n + nldf)
    return nodal + flux + vol + surf + powell + update


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg1", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the path would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wl
    from paper_1806_02343_amd import DG

    D, d, n, divb, limiter, cfg, desc = WORKLOADS[args.workload]
    field = wl.config_field(cfg)
    results = {}
    states = {}
    stream = torch.cuda.Stream()          # non-null stream: each step replays one captured hipGraph
    torch.cuda.set_stream(stream)
    for prec in ([0] if args.no_fp32 else [0, 1]):
        gpu = DG(D, d, n, divb=divb, precision=prec, limiter=limiter, cfl=0.3, stream=stream.cuda_stream)
        w0 = gpu.empty_state()
        gpu.project_field(field, w0)
        if limiter:
            gpu.limit(w0)
        variant = gpu.autotune(w0)
        w = w0.clone()
        gpu.step(w, args.warmup)
        w.copy_(w0)
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(s)
        gpu.step_async(w, args.steps)
        e1.record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        ndof = gpu.nmodes * gpu.ncells
        results[prec] = dict(ms=ms, wall=wall, ndof=ndof, value=ndof * 3 * args.steps / (ms / 1e3), gpu=gpu,
                             variant=variant)
        states[prec] = w
        # kernel timings (mean ms per launch)
        results[prec]["k_face"] = gpu.time_kernel(w0, 0, 5)
        results[prec]["k_cell"] = gpu.time_kernel(w0, 1, 5)
        results[prec]["k_dt"] = gpu.time_kernel(w0, 2, 5)
        results[prec]["k_limit"] = gpu.time_kernel(w0, 3, 5) if limiter else 0.0
        print(f"# prec={'fp64' if prec == 0 else 'fp32'} ms/step={ms / args.steps:.3f} "
              f"face={results[prec]['k_face']:.3f}ms cell={results[prec]['k_cell']:.3f}ms "
              f"dt={results[prec]['k_dt']:.3f}ms limit={results[prec]['k_limit']:.3f}ms variant={variant}",
              file=sys.stderr, flush=True)

    r64 = results[0]
    gpu = r64["gpu"]
    ncells = gpu.ncells
    # roofline of the dominant kernel (FP64)
    dom = "k_cell" if r64["k_cell"] >= r64["k_face"] else "k_face"
    flops_launch = cell_flops(D, d, divb) * ncells
    achieved = flops_launch / (r64["k_cell"] / 1e3)
    roof = {"kernel": "k_cell", "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
            "dominant": dom, "ms_per_launch": r64["k_cell"], "flops_per_launch": flops_launch}

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
                   "n_dof": r64["ndof"], "divb": "powell+ldf" if divb else "glm"},
        "roofline": roof,
    }
    if 1 in results:
        r32 = results[1]
        # FP32 state against the FP64 state of the same run (FP64 matches the oracle to 1e-12)
        a = states[1][:, :ncells].double()
        b = states[0][:, :ncells]
        rel = float((a - b).abs().sum() / b.abs().sum())
        line["fp32"] = {"value": r32["value"], "ms_per_step": r32["ms"] / args.steps,
                        "rel_l1_modal_vs_fp64": rel, "speedup_vs_fp64": r32["value"] / r64["value"]}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(D, d, divb, cfg)
    print(json.dumps(line), flush=True)


def cpu_baseline(D, d, divb, cfg):
    """The FP64 oracle timed on the host on a bounded sample of the workload:
    one SSP-RK3 step of the same scheme on a 16^3 (3-D) or 32^2 (2-D) grid."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workloads as wl
    from oracle import dg
    nsample = 16 if D == 3 else 32
    orc = dg.DG(dg.Mesh.uniform(D, nsample), d, divb=divb)
    w = orc.project(dg.conserved_field(wl.config_field(cfg), 5.0 / 3.0, orc.nvar))
    t0 = time.perf_counter()
    w, dt, ch, k = orc.step(w)
    sec = time.perf_counter() - t0
    ndof = orc.nmodes * orc.mesh.ncells
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": ndof * 3 / sec, "unit": "DoF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"1 SSP-RK3 step on {nsample}^{D} cells ({ndof} DoF), {sec:.2f} s"}


if __name__ == "__main__":
    main()
