#!/usr/bin/env python3
"""Train the conv-net preconditioner of the learned step on one GPU.

Data (all on the device, produced by the library's plain FP64 solver):
for each training potential (seeded Gaussian wells, seeds ``seed_base ..``,
disjoint from the benchmark seeds) and block width N taken in turn from
``--widths``, run plain steps of scheme (4.1) from a seeded orthonormal start
block and, at the ``--snapshots`` step counts, take the residual block
R = HU - U Lam and S = H^{-1} R (Step 1's CG at a tight tolerance).  Each
column becomes one sample: x = r / |r|, target t = s / (|r| h^2), with the
potential channel h^2 (V + shift) of its problem.

Training: Adam on the energy-norm plus residual-norm loss (default; either
alone on request, the residual loss needs no targets), each batch
``--batch`` consecutive columns of one random snapshot, cosine decay of the
learning rate.  Validation loss on held-out potentials every ``--log-every``
steps.  Writes the FP32 weights (.npy, OPE_NET_PARAMS values) and a JSON log.

    python -m paper_2511_06788_amd.train_net --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, flush=True)


def he_init(seed: int) -> np.ndarray:
    """He-normal initial weights, layer by layer ([tap][in][out])."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x7A1E]))
    out = []
    for ci, co in ((2, 16), (16, 16), (16, 16), (16, 1)):
        out.append((rng.standard_normal((27, ci, co)) * math.sqrt(2.0 / (27 * ci))).reshape(-1))
    return np.concatenate(out).astype(np.float32)


def residual_block(ope, torch, ctx, U, HU, R, Lam, Z):
    """R = HU - U Lam with Lam = U^T HU (library stencil, Gram and row update)."""
    N = ctx.N
    ope.ope_apply_h(ctx.handle, U, HU)
    ope.ope_gram(ctx.handle, U, N, N, HU, N, N, ctx.n, Lam)
    Z[:N].copy_(-Lam)
    R.copy_(U)
    ope.ope_update(ctx.handle, R, HU, Z)     # R <- U (-Lam) + HU


def harvest(ope, torch, W, problem, tau, snapshots, sample_net, solve_tol, log_prefix="", targets=True):
    """Samples (X, T) of one problem at the given step counts (device FP32, columns x n)."""
    n, N = problem.grid.n, problem.N
    ctx = ope.Context(problem.grid, problem.V, N, kinetic=problem.kinetic, shift=problem.shift)
    try:
        U = torch.from_numpy(problem.U0).cuda()
        HU = torch.empty_like(U)
        R = torch.empty_like(U)
        S = torch.empty_like(U)
        Lam = torch.empty(N, N, dtype=torch.float64, device="cuda")
        Z = torch.zeros(2 * N, N, dtype=torch.float64, device="cuda")
        Z[N:] = torch.eye(N, dtype=torch.float64, device="cuda")
        Xs, Ts = [], []
        done = 0
        for target in sorted(snapshots):
            while done < target:
                ope.ope_step(ctx.handle, U, tau)
                done += 1
            residual_block(ope, torch, ctx, U, HU, R, Lam, Z)
            its = ope.ope_source_solve(ctx.handle, R, S, None, tol=solve_tol, max_iter=20000) if targets else 0
            X = torch.empty(N, n, dtype=torch.float32, device="cuda")
            T = torch.empty_like(X)
            ope.ope_net_samples(sample_net, R, S if targets else R, N, N, X, T)
            Xs.append(X)
            Ts.append(T if targets else None)
            res, _, _ = ope.ope_residual(ctx.handle, U, N, want_ritz=False)
            log(f"{log_prefix} step {done:4d} res {res:.3e} target CG its {its}")
        return Xs, Ts
    finally:
        ctx.close()


def potential_channel(torch, problem):
    h = problem.grid.h[0]
    return torch.from_numpy((h * h * (problem.V + problem.shift)).astype(np.float32)).cuda()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--m", type=int, default=64)
    ap.add_argument("--widths", default="16,32,64,128")
    ap.add_argument("--potentials", type=int, default=32)
    ap.add_argument("--seed-base", type=int, default=1000)
    ap.add_argument("--val-seeds", default="2000,2001")
    ap.add_argument("--snapshots", default="0,4,16,48,120")
    ap.add_argument("--tau", type=float, default=45.0)
    ap.add_argument("--solve-tol", type=float, default=1e-6)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--loss", choices=["energy", "residual", "both"], default="both")
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--init", default=None, help="start from these weights (.npy)")
    ap.add_argument("--log-every", type=int, default=200)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    import torch
    import workloads as W
    from paper_2511_06788_amd import ope

    widths = [int(v) for v in args.widths.split(",")]
    snaps = [int(v) for v in args.snapshots.split(",")]
    B = args.batch
    t0 = time.time()
    # the training network lives on a context of the widest block (sample packing needs N columns)
    base = W.wells_3d(m=args.m, N=max(widths), seed=args.seed_base, with_u0=False)
    tctx = ope.Context(base.grid, base.V, base.N, kinetic=base.kinetic, shift=base.shift)
    w0 = np.load(args.init).astype(np.float32) if args.init else he_init(args.init_seed)
    net = ope.Net(tctx, B, w0)
    targets = args.loss != "residual"
    ope.ope_net_set_loss(net.handle, {"energy": ope.OPE_NET_LOSS_ENERGY, "residual": ope.OPE_NET_LOSS_RESIDUAL,
                                      "both": ope.OPE_NET_LOSS_BOTH}[args.loss])

    blocks = []     # (X, T, v2) per snapshot
    for k in range(args.potentials):
        seed = args.seed_base + k
        N = widths[k % len(widths)]
        prob = W.wells_3d(m=args.m, N=N, seed=seed)
        v2 = potential_channel(torch, prob)
        Xs, Ts = harvest(ope, torch, W, prob, args.tau, snaps, net.handle, args.solve_tol, f"train seed {seed} N {N}",
                         targets)
        blocks += [(X, T, v2) for X, T in zip(Xs, Ts)]
    val = []
    for k, seed in enumerate(int(v) for v in args.val_seeds.split(",")):
        N = [17, 64][k % 2]
        prob = W.wells_3d(m=args.m, N=N, seed=seed)
        v2 = potential_channel(torch, prob)
        Xs, Ts = harvest(ope, torch, W, prob, args.tau, [8, 60], net.handle, args.solve_tol, f"val seed {seed} N {N}",
                         targets)
        val += [(X, T, v2) for X, T in zip(Xs, Ts)]
    log(f"data: {len(blocks)} training snapshots, {sum(b[0].shape[0] for b in blocks)} columns, "
        f"{len(val)} validation snapshots, {time.time() - t0:.1f} s")

    def val_loss():
        tot, cnt = 0.0, 0
        for X, T, v2 in val:
            for k in range(0, X.shape[0] - B + 1, B):
                loss, _ = ope.ope_net_grad(net.handle, X[k:k + B], v2, T[k:k + B] if T is not None else None, B,
                                           want_grad=False)
                tot += loss
                cnt += 1
        return tot / max(cnt, 1)

    rng = np.random.default_rng(np.random.SeedSequence([args.init_seed, 0x7A1F]))
    hist = {"step": [], "train": [], "val": []}
    v0 = val_loss()
    log(f"step 0 val {v0:.4f}")
    hist["step"].append(0)
    hist["train"].append(None)
    hist["val"].append(v0)
    run = []
    t1 = time.time()
    for it in range(1, args.steps + 1):
        X, T, v2 = blocks[int(rng.integers(0, len(blocks)))]
        k = int(rng.integers(0, X.shape[0] - B + 1))
        lr = args.lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * (it - 1) / args.steps)))
        run.append(ope.ope_net_train_step(net.handle, X[k:k + B], v2, T[k:k + B] if T is not None else None, B, lr))
        if it % args.log_every == 0 or it == args.steps:
            vl = val_loss()
            tr = float(np.mean(run))
            run = []
            hist["step"].append(it)
            hist["train"].append(tr)
            hist["val"].append(vl)
            log(f"step {it} lr {lr:.2e} train {tr:.4f} val {vl:.4f} ({time.time() - t1:.1f} s)")
    w = ope.ope_net_get_weights(net.handle)
    np.save(args.out, w)
    meta = {"args": vars(args), "history": hist, "train_seconds": time.time() - t1,
            "total_seconds": time.time() - t0}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    net.close()
    tctx.close()
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
