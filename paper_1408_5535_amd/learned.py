"""Training and evaluation of the learned preconditioner on a matrix family.

The network is the message-passing preconditioner of the library (see
include/phsvds.h): it maps the residual r of a Ritz pair (theta, x) of
C = A^T A to an approximate correction for (C - theta I), a preconditioner of
the kind Section 4 admits.  The pipeline runs on the GPU through the C ABI:

  harvest   float64 stage-1 runs on the training matrices; every few
            iterations each targeted pair gets the exact solution of the
            projected equation (C - rho theta I) t = -r by conjugate
            gradients (phsvds_harvest).  The default rho = 0 (projected
            C^-1 r) gives targets a local network can approximate; with
            rho = 1 (the Jacobi-Davidson equation) the targets are dominated
            by the next eigenvectors, which three hops of message passing
            cannot represent;
  train     Adam on the mean loss ||t - t*||^2 / ||t*||^2 over mini-batches
            of harvested pairs, forward and backward by the library's
            kernels (phsvds_gnn_loss_grad, phsvds_gnn_adam);
  evaluate  k smallest triplets of held-out matrices with no
            preconditioner, with Jacobi, and with the trained network (which
            falls back to Jacobi when it stops helping), reporting products
            with A and time to a residual of tol * ||A||.

Command line (one GPU):
  python -m paper_1408_5535_amd.learned --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import DeviceCSR, GnnGraph, Solver, gnn_nweights, gnn_pack, harvest, train_gnn


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def random12(seed: int, m: int = 300_000, n: int = 200_000):
    """The random sparse family: 12 nonzeros per row at uniform random
    columns, N(0, 1) values, plus a diagonal shift U[0.01, 0.1]."""
    import workloads as wl
    return wl.random_sparse(m, n, 12, seed=seed)


def harvest_family(seeds, make, k=10, block=4, every=25, max_pairs=48, tol=1e-10,
                   cg_tol=1e-6, cg_maxit=1000, width=32, shift_scale=0.0):
    """Device matrices, prepared graphs and float32 training pairs
    (graph index, r, x, theta, t*) from stage-1 runs on each matrix."""
    mats, graphs, pairs = [], [], []
    for gi, seed in enumerate(seeds):
        t0 = time.time()
        A = DeviceCSR.from_scipy(make(seed))
        R, X, T, th, st = harvest(A, k, block=block, every=every, max_pairs=max_pairs, tol=tol,
                                  cg_tol=cg_tol, cg_maxit=cg_maxit, shift_scale=shift_scale)
        g = GnnGraph(A, width)
        mats.append(A)
        graphs.append(g)
        for j in range(R.shape[0]):
            pairs.append((gi, R[j].float().contiguous(), X[j].float().contiguous(), float(th[j]),
                          T[j].float().contiguous()))
        _say(f"[learned] harvest seed {seed}: {R.shape[0]} pairs, {st['mv_stage1']} products, "
             f"{time.time() - t0:.1f}s")
    return mats, graphs, pairs


def train(graphs, pairs, width=32, epochs=30, lr=1e-3, batch=16, seed=0):
    import workloads as wl
    w = gnn_pack(wl.gnn_init_weights(width=width, seed=seed))
    assert w.numel() == gnn_nweights(width)
    t0 = time.time()
    hist = train_gnn(graphs, pairs, w, epochs=epochs, lr=lr, batch=batch, seed=seed,
                     log=lambda s: _say(f"[learned] {s} ({time.time() - t0:.0f}s)"))
    return w, hist


def evaluate(seeds, make, w, width=32, k=10, block=4, tol=1e-12, max_matvecs=200_000,
             fallback_window=0):
    """Per held-out matrix: (method, products with A, seconds, status,
    largest residual / ||A||, fallbacks) for none, Jacobi and the network."""
    rows = []
    for seed in seeds:
        A = DeviceCSR.from_scipy(make(seed))
        for method in ("none", "jacobi", "gnn"):
            kw = {"gnn_width": width} if method == "gnn" else {}
            s = Solver(A, k, block=block, max_matvecs=max_matvecs, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sig, U, V, info = s.solve(tol, precond=method,
                                      gnn_weights=w if method == "gnn" else None,
                                      gnn_width=width, fallback_window=fallback_window)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            row = {"seed": seed, "method": method, "mv": int(info["mv_total"]),
                   "mv_prec": int(info["mv_prec"]), "seconds": dt, "status": int(info["status"]),
                   "max_res_over_norm": float(np.max(info["res"]) / info["anorm_est"]),
                   "fallbacks": int(info["fallbacks"])}
            rows.append(row)
            _say(f"[learned] eval {json.dumps(row)}")
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train-seeds", type=int, nargs=2, default=(1000, 1020))
    ap.add_argument("--eval-seeds", type=int, nargs=2, default=(2000, 2005))
    ap.add_argument("--m", type=int, default=300_000)
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--every", type=int, default=25)
    ap.add_argument("--max-pairs", type=int, default=48)
    ap.add_argument("--out", default="")
    ap.add_argument("--weights", default="", help="evaluate these weights, skip training")
    ap.add_argument("--shift-scale", type=float, default=0.0,
                    help="rho of the harvested equation (C - rho theta I) t = -r")
    args = ap.parse_args(argv)

    def make(seed):
        return random12(seed, args.m, args.n)

    if args.weights:
        w = torch.tensor(np.load(args.weights), dtype=torch.float32, device="cuda")
        hist = []
    else:
        mats, graphs, pairs = harvest_family(range(*args.train_seeds), make, every=args.every,
                                             max_pairs=args.max_pairs, width=args.width,
                                             shift_scale=args.shift_scale)
        w, hist = train(graphs, pairs, width=args.width, epochs=args.epochs)
        del mats, graphs, pairs
        torch.cuda.empty_cache()
        if args.out:
            np.save(args.out, w.cpu().numpy())
    rows = evaluate(range(*args.eval_seeds), make, w, width=args.width)
    print(json.dumps({"loss_per_epoch": hist, "evaluation": rows}), flush=True)


if __name__ == "__main__":
    main()
