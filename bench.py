#!/usr/bin/env python3
"""Benchmark: optimization iterations of periodic inverse homogenization on one GPU.

One step = one optimization iteration of the hot path on a resident cell:
density filter -> SIMP scale + multigrid hierarchy -> MG-PCG solve of the six
load cases -> C^H -> bulk-modulus sensitivities -> filter adjoint -> OC update.

Workload (default): 512^3 periodic cell, seeded Gaussian-smoothed noise
(sigma = 3*512/64 = 24 voxels) thresholded to volume fraction 0.3 with a 1e-3
floor, E0 = 1, nu = 0.3, p = 3, Emin = 1e-9, FP32 MG-PCG to relative residual
1e-6 (FP64 dot products, iterate and residual recomputation), each solve
started from the previous optimization iterate.

Prints one JSON line.  value = MG-PCG DOF-iterations per second over the timed
solves of the first form (3 n DOFs per case x PCG iterations of each case /
solve wall time); s_per_opt_iter is reported beside it.  --forms adds the
other forms of the method on the same cell (each gets its own warm-up and
steps): mixed_bf16 (bf16 multigrid vectors), mixed_bf16_stencil (also bf16
coarse stencils), learned (network warm start with the cold start as
fallback), cold (zero start every step).  By default the line carries plain
(headline), mixed_bf16, cold and learned; every form starts from the same design,
and its first-step C^H is compared with the headline form's.  The roofline object
covers the level-0 kernel with the largest share of the timed solve time of the
first form, timed with HIP events on the context stream; its HBM traffic comes
from the committed rocprofv3 counter summary when that summary was taken on the
same kernel source.  The CPU baseline times the FP64 oracle on a bounded
sample (the 64^3 box-downsample, 20 PCG iterations per load case, the six cases in
parallel worker processes).  --workload batch48 runs the batched form instead: 48 cells with sizes
drawn from {32, 48, 64, 96, 128}^3 in lockstep.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_level0_512cube.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2301_08911_amd", "csrc", f)
                  for f in ("level0.hip", "vector.hip", "hmg_internal.hpp")]


def bulk_weights():
    """dF/dC^H of F = -bulk modulus = -(1/9) sum_{i,j<3} C_ij (Voigt order 11,22,33,...)."""
    import numpy as np
    W = np.zeros((6, 6))
    W[:3, :3] = -1.0 / 9.0
    return W


def bulk_modulus(C):
    return float(C[:3, :3].sum()) / 9.0


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(paths=KERNEL_SOURCES):
    """Short digest of the level-0 kernel sources without their comments and
    blank lines (ties counter data to the code that was measured)."""
    h = hashlib.sha256()
    for p in paths:
        with open(p, encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, alg_bytes_per_launch: float):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE of launches with all six cases active, scaled by a plain copy of
    known size), if it was taken on the current level-0 source; else None.
    Launches with fewer active cases move proportionally less, so the figure is
    scaled by the algorithmic bytes of the timed launches."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k["hbm_bytes_per_launch"] * alg_bytes_per_launch / k["algorithmic_bytes_per_launch"]


def copy_bandwidth(nbytes=1 << 31, reps=5):
    """Device-to-device copy rate (read + write bytes / time), HIP events."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def _oracle_case_worker(args):
    """One load case of the oracle's FP64 block-Jacobi CG (runs in a worker process)."""
    K, f_case, iters = args
    from oracle import hmgref as O
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:  # pragma: no cover
        pass
    t0 = time.perf_counter()
    _, it, _ = O.pcg_solve(K, f_case, tol=1e-30, max_iter=iters, eps_abs=0.0)
    return int(it.sum()), time.perf_counter() - t0


def cpu_baseline(rho_full, n_full: int, sample: int, iters: int) -> dict:
    """FP64 oracle (CSR + block-Jacobi CG) timed on the host cores: the six load
    cases of the box-downsampled cell run as six worker processes, `iters` PCG
    iterations each.  Called before the GPU is touched (the workers are forked)."""
    import multiprocessing as mp
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
    workers = max(1, min(6, os.cpu_count() or 1))
    jobs = [(K, f[c:c + 1], iters) for c in range(6)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_case_worker, jobs, chunksize=1)
    dt = time.perf_counter() - t0
    dofit = float(sum(r[0] for r in res)) * 3 * sample ** 3
    return {"value": dofit / dt, "unit": "DOF-iters/s", "cores": workers, "kind": "oracle",
            "sample": f"{sample}^3 box-downsample of the benchmark cell, {iters} block-Jacobi "
                      f"PCG iterations per load case in FP64 (scipy CSR), the six cases in "
                      f"{workers} worker processes of one thread each; {dt:.1f} s wall"}


def run_form(form, x0_host, n, args, W, profile, warmup, steps):
    """Warm-up and timed optimization steps of one form; returns its record.

    Every form starts from the same design x0, so the C^H of its first step
    (whether warm-up or timed) is comparable across forms."""
    import numpy as np
    import torch
    from paper_2301_08911_amd.hmg import Context
    shape = (n, n, n)
    base = form[:-3] if form.endswith("_gs") else form
    smoother = "gs" if form.endswith("_gs") else "jacobi"
    prec = base if base.startswith("mixed_bf16") else "fp32"
    x = torch.from_numpy(x0_host.astype(np.float32).ravel()).cuda()
    rho, g, gx = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    ctx = Context(shape, precision=prec, Emin=1e-9, smoother=smoother)
    net = None
    if base == "learned":
        from paper_2301_08911_amd import nn
        net = nn.Net()
        net.load(os.path.join(ROOT, "paper_2301_08911_amd", "weights", "warmstart_l4c8.npy"))
    guesses = []
    C_first = []

    def opt_step(first):
        ctx.filter(x, out=rho, radius=2.0)
        ctx.set_density(rho)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if base == "learned":
            from paper_2301_08911_amd import nn
            rr, used = nn.warm_start(ctx, net, 0.5)
            guesses.append((round(rr, 4), used))
            init = 1
        else:
            init = 0 if (first or base == "cold") else 1
        res = ctx.solve_cases(args.tol, args.max_iter, init=init)
        ts = time.perf_counter() - t0
        C = ctx.elastic_tensor()
        ctx.sensitivity(W, out=g)
        ctx.filter(g, out=gx, radius=2.0, adjoint=True)
        ctx.oc_update(x, gx, 0.3, 0.05, 0.5, 1e-3)
        if not C_first:
            C_first.append(C)
        return res, ts, C

    for w in range(warmup):
        res, ts, C = opt_step(w == 0)
        log(f"{form} warmup {w}: iters {res.iters.tolist()} solve {ts:.3f} s B {bulk_modulus(C):.6f}")
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
    total_dofit, solve_s, iters_all, relres_max, Bs = 0.0, 0.0, [], 0.0, []
    t0 = time.perf_counter()
    for k in range(steps):
        res, ts, C = opt_step(warmup == 0 and k == 0)
        total_dofit += float(res.iters.sum()) * 3 * ctx.n
        solve_s += ts
        iters_all.append(res.iters.tolist())
        relres_max = max(relres_max, float(res.relres.max()))
        Bs.append(bulk_modulus(C))
        log(f"{form} step {k}: iters {res.iters.tolist()} relres max {res.relres.max():.2e} "
            f"solve {ts:.3f} s B {Bs[-1]:.6f} converged {res.converged}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    rec = {"dof_iters_per_s": total_dofit / solve_s if solve_s > 0 else 0.0,
           "s_per_opt_iter": elapsed / steps, "solve_s_per_opt_iter": solve_s / steps,
           "pcg_iters": iters_all, "max_relres": relres_max, "bulk_modulus": Bs,
           "precision": prec, "smoother": smoother, "warmup": warmup, "steps": steps,
           "start": {"plain": "previous iterate (zero on the first step)",
                     "mixed_bf16": "previous iterate (zero on the first step)",
                     "mixed_bf16_stencil": "previous iterate (zero on the first step)",
                     "cold": "zero", "learned": "network guess, zero if rejected"}[base],
           "C_first": C_first[0].tolist()}
    if guesses:
        rec["warm_start_relres_used"] = guesses
    prof = ctx.profile_read() if profile else None
    if profile:
        ctx.profile(False)
    levels = ctx.num_levels()
    ctx.destroy()
    return rec, prof, levels


def bench_batch(args):
    """48 cells of sizes drawn from {32, 48, 64, 96, 128}^3, solved in lockstep."""
    import numpy as np
    import torch
    from paper_2301_08911_amd import inputs as I
    from paper_2301_08911_amd.hmg import Batch
    sizes = (32, 48, 64, 96, 128)
    pick = I.uniform01(args.seed, 11, 48)
    shapes = [(sizes[int(u * 5)],) * 3 for u in pick]
    vfs = 0.1 + 0.4 * I.uniform01(args.seed, 12, 48)
    torch.cuda.set_device(0)
    b = Batch(shapes)
    t = time.perf_counter()
    for k, (s, vf) in enumerate(zip(shapes, vfs)):
        rho = I.smoothed_noise_density(s, args.seed * 100 + k, float(vf), sigma=3.0)
        b.set_density(k, torch.from_numpy(rho.astype(np.float32).ravel()).cuda())
    torch.cuda.synchronize()
    log(f"batch: {len(shapes)} cells, {sum(np.prod(s) for s in shapes)} vertices, "
        f"densities in {time.perf_counter() - t:.1f} s")
    grid, lz = b.tune()
    log(f"autotuned grid {grid}, z-chunk per cell {lz}")
    for w in range(args.warmup):
        r = b.solve(args.tol, args.max_iter)
        log(f"warmup {w}: max iters {r.iters.max()}")
    times, dofit = [], 0.0
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = b.solve(args.tol, args.max_iter)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        dofit += float(sum(r.iters[c].sum() * 3 * np.prod(shapes[c]) for c in range(len(shapes))))
        conv = int((r.relres.max(axis=1) <= args.tol).sum())
        log(f"step {k}: {times[-1]:.3f} s, max iters {r.iters.max()}, max relres "
            f"{r.relres.max():.2e}, {conv}/{len(shapes)} cells converged")
    total = sum(times)
    return {
        "metric": "MG-PCG DOF-iters/s, 48 batched cells (sizes 32-128)",
        "value": dofit / total, "unit": "DOF-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "48 periodic cells, sizes from {32,48,64,96,128}^3, smoothed noise "
                               f"sigma 3, VF U[0.1,0.5], FP32 MG-PCG to {args.tol:g} (at most "
                               f"{args.max_iter} iterations), cold start, one persistent launch "
                               "per level-0 pass, captured graphs",
                   "cells": [list(s) for s in shapes], "tuned_grid": grid, "tuned_lz": lz},
        "cells_converged": conv, "pcg_iters_per_cell": r.iters.max(axis=1).tolist(),
        "max_relres_per_cell": [float(v) for v in r.relres.max(axis=1)],
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="cells per axis")
    ap.add_argument("--forms", default="plain,plain_gs,mixed_bf16,mixed_bf16_stencil,cold,learned",
                    help="comma list of plain, mixed_bf16, mixed_bf16_stencil, learned, cold, "
                         "each optionally with the suffix _gs (eight-colour Gauss-Seidel smoother "
                         "instead of damped Jacobi) (the first is the headline and runs --warmup + --steps steps; the "
                         "others run --form-steps timed steps after one warm-up step, none for "
                         "cold and learned, whose every step starts without the previous iterate)")
    ap.add_argument("--form-steps", type=int, default=1)
    ap.add_argument("--workload", default="cell", choices=["cell", "batch48"])
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (multi-GPU "
              "sharding is a design, not built)", file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()
    if args.workload == "batch48":
        print(json.dumps(bench_batch(args)), flush=True)
        return

    import numpy as np
    from paper_2301_08911_amd import inputs as I

    n = args.n
    sigma = 3.0 * n / 64.0
    log(f"generating {n}^3 smoothed-noise cell (sigma {sigma:g}, VF 0.3)")
    t = time.perf_counter()
    x_host = I.smoothed_noise_density((n, n, n), args.seed, 0.3, sigma=sigma)
    log(f"  done in {time.perf_counter() - t:.1f} s")
    cpu = None
    if not args.no_cpu_baseline:
        # before any GPU use: the oracle's worker processes are forked
        log("timing the CPU oracle baseline")
        sample = 64 if n % 64 == 0 else n
        cpu = cpu_baseline(x_host, n, sample, 20)
        log(f"  {cpu['value']:.3e} DOF-iters/s on {cpu['cores']} cores")

    import torch
    torch.cuda.set_device(0)
    copy_gbs = copy_bandwidth()
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
    W = bulk_weights()
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    records, prof, levels = {}, None, 0
    for i, form in enumerate(forms):
        if i == 0:
            warm, steps = args.warmup, args.steps
        elif form.split("_gs")[0] in ("cold", "learned"):
            warm, steps = 0, args.form_steps
        else:
            warm, steps = 1, args.form_steps
        rec, p, L = run_form(form, x_host, n, args, W, profile=(i == 0), warmup=warm, steps=steps)
        records[form] = rec
        if i == 0:
            prof, levels = p, L
    Cref = np.array(records[forms[0]]["C_first"])
    for form, rec in records.items():
        rec["C_first_rel_diff_vs_" + forms[0]] = float(
            np.linalg.norm(np.array(rec["C_first"]) - Cref) / np.linalg.norm(Cref))
    head = records[forms[0]]

    # dominant level-0 kernel of the timed solves of the headline form
    name, (cnt, ms, by) = max(((k, v) for k, v in prof.items() if v[0] > 0),
                              key=lambda kv: kv[1][1])
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    traffic = measured_traffic(name, by / cnt) if cnt else None
    kernel_table = {k: {"launches": v[0], "ms": round(v[1], 3),
                        "GB/s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
                    for k, v in prof.items()}
    out = {
        "metric": "MG-PCG DOF-iters/s + s per opt-iter at 512^3 (learned/mixed vs plain)",
        "value": head["dof_iters_per_s"],
        "unit": "DOF-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["s_per_opt_iter"] * 1e3,
        "s_per_opt_iter": head["s_per_opt_iter"],
        "solve_s_per_opt_iter": head["solve_s_per_opt_iter"],
        "pcg_iters": head["pcg_iters"],
        "max_relres": head["max_relres"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 periodic cell, smoothed noise sigma {sigma:g} VF 0.3, "
                               f"bulk objective, {forms[0]} FP32 MG-PCG to {args.tol:g}, "
                               "filter radius 2, OC",
                   "cells": n ** 3, "levels": levels, "form": forms[0]},
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "launches": cnt, "avg_ms": ms / cnt if cnt else None,
                     "algorithmic_bytes_per_launch": by / cnt if cnt else None,
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "kernels": kernel_table,
        "forms": records,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    out["wall_s"] = time.perf_counter() - t_start
    out["fits_in_driver_run"] = out["wall_s"] < 600.0
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
