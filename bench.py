#!/usr/bin/env python3
"""Throughput of the layered-grating solver on one MI355X.

One step = one complete solve of the reduced inclusion system (sec. 5 of Lai,
Kobayashi, Barnett): GMRES from x0 = 0 to a 1e-9 relative residual, every apply
of K = I - S T + S B_phys A^+ C on the device.  Workload: the plain FP64 method
at M = 1000 (d = 1, middle layer y in [-1, 1], radii U[0.004, 0.012], indices
U[1.5, 3.0], gap 0.002, omega = 20, phi = -pi/5, P = 15), seeded and synthetic.
Setup (matrix A, its SVD, Mie, tables) is outside the timed region.

Prints one JSON line.  `roofline` is for the translation kernel (the dominant
one), timed with HIP events on the library stream during the timed solves;
`cpu_baseline` times the CPU FP64 oracle on a bounded sample of the same work.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s at 1e-9 resid, plain FP64 vs mixed+batched+warm-start; matvec %peak"
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def cpu_baseline(pb, iters, n_sample=96):
    """Oracle T-apply on a sample of target rows, extrapolated to whole solves."""
    import numpy as np
    from oracle.common import Geometry
    from oracle.multiple import apply_T_rows
    G = Geometry(pb)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(G.n_beta) + 1j * rng.standard_normal(G.n_beta)
    rows = np.linspace(0, G.M - 1, n_sample).astype(int)
    t0 = time.perf_counter()
    for a in range(0, n_sample, 8):
        apply_T_rows(G, x, rows[a:a + 8])
    t = time.perf_counter() - t0
    t_apply = t * G.M / n_sample
    return {"value": 1.0 / (iters * t_apply), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle translation apply on {n_sample} of {G.M} target rows "
                       f"({t:.1f} s, scipy AMOS Hankel, 1 thread), extrapolated to a full "
                       f"apply ({t_apply:.1f} s) x {iters} GMRES iterations; the low-rank "
                       f"layer term (<5% of the work) is not in the sample")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--restart", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {a.gpus}); "
              "a sharded solve across GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1412_7466_amd import inputs
    from paper_1412_7466_amd.grating import Context

    pb = inputs.m1000()
    ctx = Context(0)
    ctx.set_problem(pb)
    t0 = time.perf_counter()
    ctx.build()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    for _ in range(a.warmup):
        ctx.solve(tol=a.tol, restart=a.restart)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    iters = []
    resid = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        beta, st = ctx.solve(tol=a.tol, restart=a.restart)
        iters.append(st.iters)
        resid.append(st.rel_resid)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    m2l_ms, launches = ctx.profile_read()
    ctx.profile(False)
    out = ctx.bragg(beta)
    # the same workload through the mixed-precision path (FP32 translation, FP64 refinement)
    from paper_1412_7466_amd.grating import GRT_FP32
    ctx.solve(tol=a.tol, restart=a.restart, precision=GRT_FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        bm, stm = ctx.solve(tol=a.tol, restart=a.restart, precision=GRT_FP32)
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / a.steps
    mixed = {"solves_per_s": 1.0 / t_mixed, "iters": stm.iters, "refine_steps": stm.refine_steps,
             "rel_resid": stm.rel_resid,
             "rel_diff_vs_fp64": float(torch.linalg.norm(bm - beta) / torch.linalg.norm(beta))}
    P, M = pb.P, pb.M
    avg_ms = m2l_ms / max(launches, 1)
    flops = 8.0 * (2 * P + 1) ** 2 * M * M     # Toeplitz contraction per (target, source) pair
    achieved = flops / (avg_ms * 1e-3) / 1e12
    res = {
        "metric": METRIC,
        "value": a.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "m1000_fp64: plain FP64 method, M=1000, P=15, omega=20, d=1, "
                               "middle layer y in [-1,1], one angle phi=-pi/5, GMRES to 1e-9",
                   "M": M, "P": P, "n_unknowns": M * (2 * P + 1), "tol": a.tol,
                   "restart": a.restart, "seed": pb.seed},
        "gmres_iters": iters[-1],
        "rel_resid": resid[-1],
        "flux_err": out["flux_err"],
        "setup_s": t_setup,
        "mixed_fp32_fp64": mixed,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     "traffic": None, "kernel": f"m2l_kernel<{P}>",
                     "avg_launch_ms": avg_ms, "launches": launches,
                     "flops_per_launch": flops},
    }
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(pb, iters[-1])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
