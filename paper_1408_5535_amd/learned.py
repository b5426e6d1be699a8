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
  init      the network starts as the polynomial preconditioner
            D^-1/2 p(Ch) D^-1/2 with p a degree-3 least-squares fit of 1/x on
            (0, 1.05 ||A D^-1/2||^2] (the norm from the library's own
            largest-mode solve), written into the weights (channels carry
            the positive and negative parts of Ch^k u); or as exactly the
            Jacobi preconditioner (--init jacobi: Glorot layers, zero
            readout); or from Glorot weights (--init glorot);
  train     Adam on the mean loss over mini-batches of harvested pairs,
            forward and backward by the library's kernels: by default
            ||C t - r||^2 / ||r||^2, how far the correction is from solving
            C t = r (phsvds_gnn_residual_loss_grad), the criterion the
            polynomial start fits, here weighted by the residuals the
            iteration produces; or (--loss target) ||t - t*||^2 / ||t*||^2,
            the distance to the exact corrections (phsvds_gnn_loss_grad),
            which the lowest modes dominate and a three-hop network cannot
            follow: it trains the network away from good preconditioners;
  select    among the start and the checkpoints at a quarter, half and
            the end of training, the network with the fewest products on a
            validation matrix (neither loss is the quality inside the
            iteration itself);
  evaluate  k smallest triplets of held-out matrices with no
            preconditioner, with Jacobi, with the network at its start, the
            last checkpoint and the selected one (each falls back to Jacobi
            when it stops helping), reporting products with A and time to a
            residual of tol * ||A||.

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
        # the harvested targets are M r with M ~ (projected C - rho theta)^-1,
        # the sign of the Jacobi step the network starts from
        for j in range(R.shape[0]):
            pairs.append((gi, R[j].float().contiguous(), X[j].float().contiguous(), float(th[j]),
                          T[j].float().contiguous()))
        _say(f"[learned] harvest seed {seed}: {R.shape[0]} pairs, {st['mv_stage1']} products, "
             f"{time.time() - t0:.1f}s")
    return mats, graphs, pairs


def ch_norm_bound(A_host):
    """||A D^-1/2||^2 = the largest eigenvalue of Ch = D^-1/2 A^T A D^-1/2
    (D = diag(A^T A)): the scaling and the largest-mode solve (k = 1) both
    run in the library."""
    from . import jacobi_scaled, svds_smallest
    B = jacobi_scaled(DeviceCSR.from_scipy(A_host))
    sig, _, _, info = svds_smallest(B, 1, 1e-10, which="largest", block=1)
    return float(sig[0]) ** 2


def poly_init(A_host, width=32, degree=3, margin=1.05):
    """Initial weights: the polynomial preconditioner D^-1/2 p(Ch) D^-1/2,
    p fitted to 1/x on (0, margin ||A D^-1/2||^2]."""
    import workloads as wl
    hi = margin * ch_norm_bound(A_host)
    coeffs = wl.inverse_poly_coeffs(hi, degree)
    return gnn_pack(wl.gnn_poly_weights(coeffs, width)), hi, coeffs


def jacobi_init(width=32, seed=0):
    """Initial weights whose network is exactly the Jacobi preconditioner:
    Glorot layers and a zero readout (the readout adds the Jacobi feature),
    so training starts from Jacobi with live hidden channels."""
    import workloads as wl
    P = wl.gnn_init_weights(width=width, seed=seed)
    P["wo"][:] = 0.0
    return gnn_pack(P)


def train(graphs, pairs, width=32, epochs=30, lr=1e-3, batch=16, seed=0, init=None,
          checkpoints=(), loss_kind="residual"):
    """Adam from `init` (or Glorot weights); returns (final weights, loss per
    epoch, {epoch: weights} for the epochs in `checkpoints`)."""
    import workloads as wl
    w = (init.clone() if init is not None
         else gnn_pack(wl.gnn_init_weights(width=width, seed=seed)))
    assert w.numel() == gnn_nweights(width)
    t0 = time.time()
    snaps = {}

    def keep(ep, cur):
        if ep in checkpoints:
            snaps[ep] = cur.clone()

    hist = train_gnn(graphs, pairs, w, epochs=epochs, lr=lr, batch=batch, seed=seed,
                     log=lambda s: _say(f"[learned] {s} ({time.time() - t0:.0f}s)"),
                     on_epoch=keep, loss_kind=loss_kind)
    return w, hist, snaps


def select_by_validation(cands, make, seed, width=32, k=10, block=4):
    """The candidate network (name -> weights) with the fewest products with
    A on one validation matrix (ties: the first), and the products of each.
    The training loss measures the distance to exact corrections, which is
    not what makes a preconditioner good inside the iteration; the
    validation solve measures that directly."""
    rows = evaluate([seed], make, cands, width=width, k=k, block=block, baselines=False)
    mv = {r["method"]: r["mv"] for r in rows if r["status"] == 0}
    best = min(mv, key=lambda name: (mv[name], list(cands).index(name))) if mv else list(cands)[0]
    return best, {r["method"]: (r["mv"], r["status"]) for r in rows}


def evaluate(seeds, make, nets, width=32, k=10, block=4, tol=1e-12, max_matvecs=200_000,
             fallback_window=0, baselines=True):
    """Per held-out matrix: (method, products with A, seconds, status,
    largest residual / ||A||, fallbacks) for none, Jacobi and each network
    (``nets``: name -> weights, or one weight tensor named 'gnn')."""
    if isinstance(nets, torch.Tensor):
        nets = {"gnn": nets}
    rows = []
    for seed in seeds:
        A = DeviceCSR.from_scipy(make(seed))
        for method in (["none", "jacobi"] if baselines else []) + list(nets):
            net = nets.get(method)
            kw = {"gnn_width": width} if net is not None else {}
            s = Solver(A, k, block=block, max_matvecs=max_matvecs, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sig, U, V, info = s.solve(tol, precond="gnn" if net is not None else method,
                                      gnn_weights=net, gnn_width=width,
                                      fallback_window=fallback_window)
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
    ap.add_argument("--family", choices=["random", "powerlaw"], default="random",
                    help="random: 12 per row at uniform columns; powerlaw: shifted Zipf(2) row "
                         "lengths with mean 10 and at most 2000 (both with the diagonal shift)")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--block", type=int, default=4)
    ap.add_argument("--max-mv", type=int, default=200_000,
                    help="product budget of each evaluation solve")
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
    ap.add_argument("--init", choices=["poly", "jacobi", "glorot"], default="poly",
                    help="polynomial preconditioner, Jacobi (Glorot layers, zero readout), "
                         "or Glorot weights")
    ap.add_argument("--val-seed", type=int, default=1500,
                    help="validation matrix for choosing among the checkpoints")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--loss", choices=["target", "residual"], default="residual",
                    help="distance to the exact corrections, or ||C t - r|| / ||r||")
    args = ap.parse_args(argv)

    def make(seed):
        if args.family == "powerlaw":
            import workloads as wl
            return wl.powerlaw_sparse(args.m, args.n, seed=seed)
        return random12(seed, args.m, args.n)

    nets, meta = {}, {}
    if args.weights:
        nets["gnn"] = torch.tensor(np.load(args.weights), dtype=torch.float32, device="cuda")
        hist = []
    else:
        init = None
        if args.init == "poly":
            init, hi, coeffs = poly_init(make(args.train_seeds[0]), args.width)
            nets["gnn_init"] = init
            meta = {"ch_bound": hi, "poly_coeffs": [float(c) for c in coeffs]}
            _say(f"[learned] polynomial start: bound {hi:.4f}, coefficients {meta['poly_coeffs']}")
        elif args.init == "jacobi":
            init = jacobi_init(args.width)
            nets["gnn_init"] = init
        # the residual objective needs no exact corrections: no CG
        mats, graphs, pairs = harvest_family(range(*args.train_seeds), make, every=args.every,
                                             max_pairs=args.max_pairs, width=args.width,
                                             shift_scale=args.shift_scale,
                                             cg_maxit=0 if args.loss == "residual" else 1000)
        marks = sorted({args.epochs // 4 - 1, args.epochs // 2 - 1, args.epochs - 1} - {-1})
        w, hist, snaps = train(graphs, pairs, width=args.width, epochs=args.epochs, lr=args.lr,
                               init=init, checkpoints=marks, loss_kind=args.loss)
        del mats, graphs, pairs
        torch.cuda.empty_cache()
        # checkpoint selection on a validation matrix (not a training or
        # evaluation seed)
        cands = ({"start": init} if init is not None else {})
        cands.update({f"epoch{e + 1}": snaps[e] for e in marks})
        best, val = select_by_validation(cands, make, args.val_seed, width=args.width, k=args.k,
                                         block=args.block)
        meta["validation"] = {name: v[0] for name, v in val.items()}
        meta["selected"] = best
        _say(f"[learned] validation products {meta['validation']}, selected {best}")
        nets["gnn_last"] = w
        nets["gnn"] = cands[best]
        if args.out:
            np.save(args.out, cands[best].cpu().numpy())
    rows = evaluate(range(*args.eval_seeds), make, nets, width=args.width, k=args.k,
                    block=args.block, max_matvecs=args.max_mv)
    print(json.dumps({"loss_per_epoch": hist, "init": meta, "evaluation": rows}), flush=True)


if __name__ == "__main__":
    main()
