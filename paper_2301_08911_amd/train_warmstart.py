"""Train the learned warm start on solver-generated data (GPU only).

Data: seeded smoothed-noise cells (volume fraction ~ U[0.1, 0.5], sigma = 3
voxels, 1e-3 floor) filtered with the radius-2 density filter, solved with the
FP32 MG-PCG; the pair is (filtered density, u / N) on the cell's grid, or on
its multigrid level of size 64 for larger cells (density box mean, u at the
coarse vertices).  The network, its forward/backward kernels and Adam are the
library's own (include/hmg_nn.h); this script only drives them.

    python -m paper_2301_08911_amd.train_warmstart --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import inputs as I
from .hmg import Context
from .nn import Net, warm_start

TRAIN_STREAM = 7  # seeds of training cells are (base + k); held-out cells use another base


def make_cell(n, seed):
    """Filtered smoothed-noise density of an n^3 cell and its volume fraction."""
    vf = 0.1 + 0.4 * float(I.uniform01(seed, 9, 1)[0])
    x = I.smoothed_noise_density((n, n, n), seed, vf, sigma=3.0).astype(np.float32).ravel()
    return x, vf


def solve_pair(n, seed, tol, dim_out=64):
    """(input [1, D^3], target [18, D^3]) for one cell, D = min(n, dim_out)."""
    x, _ = make_cell(n, seed)
    ctx = Context((n, n, n), precision="fp32")
    xd = torch.from_numpy(x).cuda()
    rho = ctx.filter(xd, radius=2.0)
    ctx.set_density(rho)
    res = ctx.solve_cases(tol, 2000)
    u = ctx.get_displacement()  # (6, 3, n^3) float32
    f = n // min(n, dim_out)
    D = n // f
    rho3 = rho.view(n, n, n)
    u5 = u.view(18, n, n, n)
    if f > 1:
        rho3 = rho3.view(D, f, D, f, D, f).mean(dim=(1, 3, 5))
        u5 = u5[:, ::f, ::f, ::f]
    inp = rho3.reshape(1, D, D, D).contiguous()
    tgt = (u5 / n).reshape(18, D, D, D).contiguous()
    del ctx
    return inp, tgt, res.iters.max()


def generate(sizes, counts, base_seed, tol, log):
    data = {}
    for n, cnt in zip(sizes, counts):
        xs, ys = [], []
        t0 = time.perf_counter()
        for k in range(cnt):
            inp, tgt, it = solve_pair(n, base_seed + 1000 * n + k, tol)
            xs.append(inp)
            ys.append(tgt)
            if (k + 1) % 100 == 0:
                log(f"  {k + 1} of {cnt} cells of {n}^3 ({time.perf_counter() - t0:.1f} s)")
        D = xs[0].shape[-1]
        data[D] = data.get(D, ([], []))
        data[D][0].extend(xs)
        data[D][1].extend(ys)
        log(f"generated {cnt} cells of {n}^3 in {time.perf_counter() - t0:.1f} s")
    return {D: (torch.stack(a), torch.stack(b)) for D, (a, b) in data.items()}


def train(net, data, steps, batch, lr, log):
    keys = sorted(data)
    rng = np.random.default_rng(0)
    tot = sum(data[D][0].shape[0] for D in keys)
    dys, ys = {}, {}
    losses = []
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        # pick a resolution group in proportion to its size, then a batch
        D = keys[int(rng.choice(len(keys), p=[data[k][0].shape[0] / tot for k in keys]))]
        X, Y = data[D]
        idx = torch.from_numpy(rng.choice(X.shape[0], size=min(batch, X.shape[0]), replace=False))
        xb = X[idx.cuda()].contiguous()
        tb = Y[idx.cuda()].contiguous()
        key = (D, xb.shape[0])
        if key not in ys:
            ys[key] = torch.empty_like(tb)
            dys[key] = torch.empty_like(tb)
        net.forward(xb, out=ys[key])
        loss = net.mse(ys[key], tb, dys[key])
        net.zero_grad()
        net.backward(dys[key])
        cur = lr * 0.5 * (1 + math.cos(math.pi * (step - 1) / steps))  # cosine decay
        net.adam_step(cur, step)
        losses.append(loss)
        if step % max(1, steps // 20) == 0:
            log(f"step {step}: loss {np.mean(losses[-50:]):.3e} ({time.perf_counter() - t0:.1f} s)")
    return losses


def evaluate(net, sizes, base_seed, tol, accept, log):
    """Cold start vs learned start on held-out cells.  The learned start spends
    one multigrid cycle on its correction; `zero_relres` is what that single
    cycle reaches from u = 0, the baseline the prediction has to beat."""
    zero = Net(seed=1)
    zero.set_params(np.zeros(zero.param_count, np.float32))
    out = []
    for n in sizes:
        x, vf = make_cell(n, base_seed + n + len(out))
        xd = torch.from_numpy(x).cuda()
        cold = Context((n, n, n), precision="fp32")
        rho = cold.filter(xd, radius=2.0)
        cold.set_density(rho)
        rc = cold.solve_cases(tol, 3000)
        probe = Context((n, n, n), precision="fp32")
        probe.set_density(rho)
        zr, _ = warm_start(probe, zero, 0.0)
        del probe
        warm = Context((n, n, n), precision="fp32")
        warm.set_density(rho)
        rr, used = warm_start(warm, net, accept)
        rw = warm.solve_cases(tol, 3000, init=1)
        rec = {"n": n, "vf": vf, "cold_iters": rc.iters.tolist(), "guess_relres": rr,
               "zero_relres": zr, "used": used,
               "warm_iters": (rw.iters + (1 if used else 0)).tolist()}
        log(json.dumps(rec))
        out.append(rec)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--cells32", type=int, default=256)
    ap.add_argument("--cells64", type=int, default=96)
    ap.add_argument("--cells128", type=int, default=16)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)

    def log(msg):
        print(f"[train] {msg}", flush=True)

    torch.cuda.set_device(0)
    data = generate((32, 64, 128), (args.cells32, args.cells64, args.cells128),
                    100000 * TRAIN_STREAM, args.tol, log)
    net = Net(seed=args.seed)
    log(f"network: {net.param_count} parameters; groups "
        f"{ {D: int(v[0].shape[0]) for D, v in data.items()} }")
    losses = train(net, data, args.steps, args.batch, args.lr, log)
    net.save(args.out)
    meta = {"levels": 4, "base_channels": 8, "in_channels": 1, "out_channels": 18,
            "cells": [args.cells32, args.cells64, args.cells128], "steps": args.steps,
            "batch": args.batch, "lr": args.lr, "final_loss": float(np.mean(losses[-100:]))}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    evaluate(net, (64, 64, 128, 128), 900000, 1e-6, 0.5, log)


if __name__ == "__main__":
    sys.exit(main())
