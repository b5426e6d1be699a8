"""Dynamic switching between the normal equations and the augmented
matrix (Section 4.1, Algorithm 3), float64.  Test infrastructure: the CPU
oracle of the GPU path's dynamic mode, not part of the product.

With a preconditioner whose strength on C = A^T A and on B = [0 A^T; A 0]
is not known, short GD+k runs alternate between the two, each starting
from the other's latest approximations, and the measured convergence rates
decide which approach finishes the solve.  Readings (the paper gives the
rules, not every constant):
  * a run's rate is the mean, over its iterations, of the factor by which
    the residual of the leading unconverged target fell from one iteration
    to the next; iterations where the target changed (a lock) start a new
    segment.  A C run measures ||r_C|| / sigma, a B run ||r_B|| (each the
    size of the triplet residual up to a constant), so rates compare;
  * initIter = 50 and maxSwitch = 8; both approaches run GD+k;
  * a B run targets the current estimates of the k smallest singular values
    with seeds [v; A v / ||A v||] (a random left vector where A v carries no
    accuracy, as in the transition);
  * numConverged adds up the pairs each run locked;
  * B runs take harmonic Ritz vectors for the target 0 (the smallest
    positive eigenvalues of B with balanced halves): the estimates of a
    short run are too rough to serve as the refined projection's shifts,
    and a shift far above sigma_1 would converge to another singular value;
  * once decided, the chosen approach finishes the solve from the latest
    approximations of all k pairs: C -> the two-stage method with them as
    its initial basis; B -> GD+k on B as in the switching runs, without an
    iteration limit.  A run that locked all k pairs ends the switching the
    same way (its pairs lock again at once).
Pinned: the control loop against hand-traced runs, the extraction, and the
results against closed forms.  Parity unpinned: the measured rates, which
move with rounding; where the two approaches' rates lie close the GPU's
later runs may differ from these.
"""
from __future__ import annotations

import math

import numpy as np

from . import phsvds as ph

INIT_ITER = 50
MAX_SWITCH = 8


def segment_rate(logs):
    """exp of the mean one-step change of log residual, over consecutive
    entries of the same segment (None separates segments); 1.0 when no step
    was measured."""
    d = [b - a for a, b in zip(logs, logs[1:]) if a is not None and b is not None]
    return math.exp(sum(d) / len(d)) if d else 1.0


def switch_control(run, k, init_iter=INIT_ITER, max_switch=MAX_SWITCH):
    """Algorithm 3's decisions.  ``run(approach, max_iter)`` runs GD+k on
    'C' or 'B' from the latest approximations for at most max_iter
    iterations and returns (rate, pairs locked in the run).  Returns
    (final approach, how: 'found' when a run locked all k pairs, else
    'faster', the list of (approach, max_iter, rate, locked) runs)."""
    runs = []
    rates = {}
    num_conv = 0
    for ap in ("C", "B"):
        rate, c = run(ap, init_iter)
        runs.append((ap, init_iter, rate, c))
        rates[ap] = rate
        num_conv += c
        if c >= k:
            return ap, "found", runs
    num_switch, j = 0, 0
    last = "B"
    while num_switch < max_switch:
        choice = "C" if rates["C"] <= rates["B"] else "B"
        if (num_switch == 0 and num_conv > 0) or num_conv > 1:
            break
        j = j + 1 if choice == last else j // 2
        max_iter = init_iter * 2 ** j
        num_switch += 1
        rate, c = run(choice, max_iter)
        runs.append((choice, max_iter, rate, c))
        rates[choice] = rate
        num_conv += c
        last = choice
        if c >= k:
            return choice, "found", runs
    return ("C" if rates["C"] <= rates["B"] else "B"), "faster", runs


def phsvds_dynamic(A, k, tol=1e-12, block=1, precond="none", anorm=None, init_iter=INIT_ITER,
                   max_switch=MAX_SWITCH, seed=2, stage2_method="jdqmr", max_restarts=10000):
    """The k smallest singular triplets with Algorithm 3 choosing the
    approach.  ``precond`` as for phsvds: 'none', 'jacobi', or
    ('inverse_A', Minv, MinvT) for M ~ A.  Returns phsvds's dict plus
    'dynamic': {choice, how, runs}; products of the switching runs are
    included in the stats."""
    import workloads  # seeded inputs only

    m, n = A.shape
    b = block
    stats = ph.Stats()
    pmax, pmin = ph.basis_sizes(k, b, n=n)
    if isinstance(precond, tuple) and precond[0] == "inverse_A":
        pc1, pcB = ph.approx_A_forms(precond[1], precond[2], n)
    elif precond == "jacobi":
        d = ph.jacobi_diag(A)
        pc1, pcB = ph.jacobi_precond_C(d), ph.jacobi_precond_B(A, d, stats)
    elif precond == "none":
        pc1 = pcB = None
    else:
        raise ValueError(precond)
    an = float(anorm) if anorm else math.sqrt(ph._power_norm2(A, seed, stats))
    st = {"V": workloads.initial_block(n, b, seed), "sig": None}

    def run_C(iters):
        logs, key = [], [None]

        def cb(it, X, R, theta, Xl):
            s0 = math.sqrt(max(float(theta[0]), 1e-300))
            if key[0] is not None and Xl.shape[1] != key[0]:
                logs.append(None)
            key[0] = Xl.shape[1]
            logs.append(math.log(max(float(np.linalg.norm(R[:, 0])) / s0, 1e-300)))

        V0 = st["V"]
        X0 = V0[:, :max(1, min(V0.shape[1], k))]
        Xl, thl, _, _, info = ph.stage1_gdk(A, k, tol, b, pmax, pmin, X0, precond=pc1,
                                            anorm=an, max_iters=iters, callback=cb, stats=stats,
                                            max_restarts=max_restarts)
        bth, bX = info["best"]
        th = np.concatenate([np.asarray(thl, dtype=np.float64), bth])
        Xa = np.column_stack([Xl, bX])
        o = np.argsort(th, kind="stable")
        st["V"], st["sig"] = Xa[:, o], np.sqrt(np.maximum(th[o], 0.0))
        return segment_rate(logs), len(thl)

    def run_B(iters):
        sig = st["sig"]
        v0 = st["V"][:, :k]
        v0 = v0 / np.linalg.norm(v0, axis=0)
        u0 = A @ v0
        stats.mv_rr += k
        nu = np.linalg.norm(u0, axis=0)
        u0 = ph._random_tiny_left(u0 / np.where(nu > 0, nu, 1.0), sig, an, ph._Rand(seed + 11))
        trace, best = [], []
        th2, X2 = ph.stage2_refined(A, sig, v0, u0, tol, an, b, pmax, pmin, pcB, max_restarts,
                                    stats=stats, max_iters=iters, method="gdk", trace=trace,
                                    best=best, extract="harmonic0")
        logs, prev = [], None
        for (_, _, _, rn, _, shift) in trace:
            if prev is not None and shift != prev:
                logs.append(None)
            prev = shift
            logs.append(math.log(max(rn, 1e-300)))
        xs = [X2[:, i] for i in range(X2.shape[1])] + [x for _, x in best]
        ss = np.abs(np.asarray(list(th2) + [t for t, _ in best], dtype=np.float64))
        Va = np.column_stack([x[:n] / np.linalg.norm(x[:n]) for x in xs])
        o = np.argsort(ss, kind="stable")
        st["V"], st["sig"] = Va[:, o], ss[o]
        return segment_rate(logs), X2.shape[1]

    choice, how, runs = switch_control(lambda ap, it: run_C(it) if ap == "C" else run_B(it), k,
                                       init_iter, max_switch)
    kw = dict(block=b, precond=precond, anorm=an, seed=seed, stage2_method=stage2_method,
              max_restarts=max_restarts)
    if choice == "C":
        out = ph.phsvds(A, k, tol, init_V=st["V"][:, :k], **kw)
    else:
        kw["stage2_method"] = "gdk"
        out = ph.phsvds(A, k, tol, init_V=st["V"][:, :k], shifts=st["sig"][:k],
                        stage2_extract="harmonic0", **kw)
    fin = out["stats"]
    for f in ("mv_stage1", "mv_rr", "mv_stage2", "mv_final", "mv_prec", "iters1", "iters2",
              "inner2"):
        setattr(fin, f, getattr(fin, f) + getattr(stats, f))
    out["dynamic"] = {"choice": choice, "how": how, "runs": runs}
    return out
