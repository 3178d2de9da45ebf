#!/usr/bin/env python3
"""Benchmark: optimization iterations of periodic inverse homogenization on one GPU.

One step = one optimization iteration of the hot path on a resident cell:
density filter -> SIMP scale + multigrid hierarchy -> MG-PCG solve of the six
load cases (warm-started from the previous iterate) -> C^H -> bulk-modulus
sensitivities -> filter adjoint -> OC update.

Workload (default): 512^3 periodic cell, seeded Gaussian-smoothed noise
(sigma = 3*512/64 = 24 voxels) thresholded to volume fraction 0.3 with a 1e-3
floor, E0 = 1, nu = 0.3, p = 3, Emin = 1e-9, FP32 MG-PCG to relative residual
1e-6 (FP64 dot products, iterate and residual recomputation).

Prints one JSON line.  value = MG-PCG DOF-iterations per second over the timed
solves (3 n DOFs per case x PCG iterations of each case / solve wall time);
s_per_opt_iter is reported beside it.  The roofline object covers the level-0
kernel with the largest share of the timed solve time, timed with HIP events
on the context stream; the CPU baseline times the FP64 oracle on a bounded
sample (a box-downsampled copy of the same cell, a fixed number of PCG
iterations).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(rho_full, n_full: int, sample: int, iters: int) -> dict:
    """FP64 oracle (CSR + block-Jacobi CG) timed on the host for `iters` PCG iterations."""
    import numpy as np
    from oracle import hmgref as O
    from paper_2301_08911_amd import inputs as I
    factor = n_full // sample
    rho = I.box_downsample(rho_full, factor)
    shape = (sample, sample, sample)
    K0, chi = O.element_stiffness(), O.unit_strain_displacements()
    s = O.simp_scale(rho)
    K = O.assemble_stiffness(s, shape, K0)
    f = O.load_vectors(s, shape, K0, chi)
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(1)
    except ImportError:  # pragma: no cover
        limit = None
    t0 = time.perf_counter()
    _, it, _ = O.pcg_solve(K, f, tol=1e-30, max_iter=iters, eps_abs=0.0)
    dt = time.perf_counter() - t0
    if limit is not None:
        limit.restore_original_limits()
    dofit = float(np.sum(it)) * 3 * sample ** 3
    return {"value": dofit / dt, "unit": "DOF-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}^3 box-downsample of the benchmark cell, {iters} block-Jacobi PCG "
                      f"iterations x 6 cases in FP64 (scipy CSR, one thread); {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="cells per axis")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported by this build "
              "(multi-GPU sharding is design-only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from oracle import hmgref as O
    from paper_2301_08911_amd import inputs as I
    from paper_2301_08911_amd.hmg import Context

    torch.cuda.set_device(0)
    n = args.n
    shape = (n, n, n)
    sigma = 3.0 * n / 64.0
    log(f"generating {n}^3 smoothed-noise cell (sigma {sigma:g}, VF 0.3)")
    t = time.perf_counter()
    x_host = I.smoothed_noise_density(shape, args.seed, 0.3, sigma=sigma)
    log(f"  done in {time.perf_counter() - t:.1f} s")
    x = torch.from_numpy(x_host.astype(np.float32).ravel()).cuda()
    rho = torch.empty_like(x)
    g = torch.empty_like(x)
    gx = torch.empty_like(x)
    W = O.bulk_weights()
    ctx = Context(shape, precision=args.precision, Emin=1e-9)
    log(f"context: {ctx.num_levels()} levels, omega {[round(ctx.level_omega(l), 3) for l in range(ctx.num_levels())]}")

    def opt_step(init):
        ctx.filter(x, out=rho, radius=2.0)
        ctx.set_density(rho)
        t0 = time.perf_counter()
        res = ctx.solve_cases(args.tol, args.max_iter, init=init)
        ts = time.perf_counter() - t0
        C = ctx.elastic_tensor()
        ctx.sensitivity(W, out=g)
        ctx.filter(g, out=gx, radius=2.0, adjoint=True)
        ctx.oc_update(x, gx, 0.3, 0.05, 0.5, 1e-3)
        return res, ts, C

    for w in range(args.warmup):
        res, ts, C = opt_step(0 if w == 0 else 1)
        log(f"warmup {w}: iters {res.iters.tolist()} relres max {res.relres.max():.2e} solve {ts:.3f} s "
            f"B {O.bulk_modulus(C):.5f}")
    torch.cuda.synchronize()
    ctx.profile(True)
    total_dofit = 0.0
    solve_s = 0.0
    iters_all = []
    relres_max = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        res, ts, C = opt_step(0 if (args.warmup == 0 and k == 0) else 1)
        total_dofit += float(res.iters.sum()) * 3 * ctx.n
        solve_s += ts
        iters_all.append(res.iters.tolist())
        relres_max = max(relres_max, float(res.relres.max()))
        log(f"step {k}: iters {res.iters.tolist()} relres max {res.relres.max():.2e} solve {ts:.3f} s "
            f"B {O.bulk_modulus(C):.5f} converged {res.converged}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)

    # dominant level-0 kernel of the timed solves
    name, (cnt, ms, by) = max(((k, v) for k, v in prof.items() if v[0] > 0),
                              key=lambda kv: kv[1][1])
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    kernel_table = {k: {"launches": v[0], "ms": round(v[1], 3),
                        "GB/s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
                    for k, v in prof.items()}
    value = total_dofit / solve_s if solve_s > 0 else 0.0
    out = {
        "metric": "MG-PCG DOF-iters/s + s per opt-iter at 512^3 (learned/mixed vs plain)",
        "value": value,
        "unit": "DOF-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "s_per_opt_iter": elapsed / args.steps,
        "solve_s_per_opt_iter": solve_s / args.steps,
        "pcg_iters": iters_all,
        "max_relres": relres_max,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 periodic cell, smoothed noise sigma {sigma:g} VF 0.3, "
                               f"bulk objective, {args.precision.upper()} MG-PCG to {args.tol:g}, "
                               "warm start from the previous iterate, filter radius 2, OC",
                   "cells": n ** 3, "levels": ctx.num_levels(), "precision": args.precision},
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "launches": cnt, "avg_ms": ms / cnt if cnt else None,
                     "algorithmic_bytes_per_launch": by / cnt if cnt else None},
        "kernels": kernel_table,
    }
    if not args.no_cpu_baseline:
        sample = 32 if n >= 32 else n
        log("timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(x_host, n, sample, 120)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
