"""Two-stage PHSVDS, float64, written step by step from the paper.

Notation follows the paper: A is m x n (m >= n, full column rank),
C = A^T A (eigenpairs (sigma_i^2, v_i)), B = [0 A^T; A 0] acting on [v; u]
(eigenpairs (+-sigma_i, [v_i; +-u_i]) and m - n zeros), Section 1.

Stage 1 (Algorithm 1): block GD+k on C for the k smallest (or largest)
eigenpairs, stopped per pair by the dynamic tolerance of Section 3.1,
    ||r_C|| < max(delta * s_i * s_n, floor * eps * s_n^2),
where s_i is the targeted Ritz value's square root and s_n^2 the largest
Ritz value seen so far (the running estimate of ||C||, Algorithm 1).

Transition (Section 3.1, Algorithm 1 step 3): a complete Rayleigh-Ritz on C
over the converged vectors plus the leading restart basis; it gives the
shifts and initial vectors [v_i; A v_i / ||A v_i||] of stage 2, with a random
left vector when sigma_i is too small to carry any accuracy (Section 3.3).

Stage 2 (Algorithm 2): GD+k on B with the refined projection: for the
current target shift s, the refined vector y minimises ||(W - s V) y|| over
the search space through the R factor of W - s V; theta = y^T H y replaces
the Ritz value; converged pairs are locked and the next initial guess is
re-inserted; corrections are t = Prec(r).

Readings where the paper is silent (the same readings bind the GPU path):
  * basis sizes: p_max = min(64, max(35, 2k + 2b)), p_min = max(21,
    ceil(0.6 p_max)), and p_min <= p_max - 2b (the paper's 35/21 for blocks
    of 1-2); locked vectors leave the basis, so k may exceed p_max;
  * GD+k restart keeps the p_min lowest Ritz vectors plus the previous
    iteration's b targeted Ritz vectors, orthogonalised against them (a
    dependent one is replaced by an independent coordinate vector of the
    coefficient space, so the restarted basis always has p_min + b columns);
  * hard locking in both stages; only the first (k - locked) targets of the
    block are tested for convergence; in stage 1 a pair that passes the test
    on its recurrence residual W s - theta x is locked only if its explicit
    residual C x - theta x passes too (one product per candidate); otherwise
    W = C V and H are recomputed to remove the drift of the restarts, at
    most once in 10 iterations (in between, a failed check just means no
    lock in that iteration: near the floor the two residuals differ by
    rounding and could otherwise alternate for ever);
  * floor = 10 in the stage-1 test; a pair whose test is floor-limited, whose
    residual is within 10x of that floor and has not improved by 10% over
    the last L = max(100, 20 p_max / b) iterations is accepted as converged
    to the floor (a guard against endless stagnation at rounding level);
  * stage 2 is entered for the pairs whose stage-1 test was floor-limited,
    i.e. delta * s_i < floor * eps * s_n (Section 3.1);
  * the transition Rayleigh-Ritz over an orthonormal Z is evaluated as the
    SVD of A Z (Z^T C Z = (AZ)^T (AZ)), which yields the same Ritz pairs of C
    without squaring the small singular values;
  * the Krylov fill of stage 2 starts from [v_1; u_1] / sqrt(2) and has
    dimension p_min - k (Algorithm 2 step 2);
  * block members 2..b of stage 2 are the next right singular vectors of R,
    accepted only if theta > s / 2 and the two halves have balanced norms;
  * dependent columns (norm drop by more than 1e10 under orthogonalisation)
    are replaced by counter-based random vectors.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import jdqmr as _jd
from . import rng as _rng

EPS64 = 2.0 ** -52
DEP_DROP = 1e-10


def basis_sizes(k: int, b: int, max_basis: int | None = None, min_restart: int | None = None,
                n: int | None = None):
    """(p_max, p_min): p_max = min(64, max(35, 2k + 2b)) capped at n (a basis
    cannot outgrow the space), p_min = max(21, ceil(0.6 p_max)) capped at
    p_max - 2b; p_min must hold a block (so n >= 3b)."""
    pmax = max_basis if max_basis else min(64, max(35, 2 * k + 2 * b))
    if n is not None:
        pmax = min(pmax, n)
    pmin = min_restart if min_restart else max(21, int(math.ceil(0.6 * pmax)))
    pmin = min(pmin, pmax - 2 * b)
    if pmin < b:
        raise ValueError("basis too small for the block size")
    return pmax, pmin


@dataclass
class Stats:
    mv_stage1: int = 0
    mv_rr: int = 0
    mv_stage2: int = 0
    mv_final: int = 0
    mv_prec: int = 0
    iters1: int = 0
    iters2: int = 0
    restarts1: int = 0
    restarts2: int = 0
    inner2: int = 0
    stage2_pairs: int = 0
    fallback: bool = False
    anorm_est: float = 0.0
    res_stage1: list = field(default_factory=list)

    @property
    def mv_total(self):
        return self.mv_stage1 + self.mv_rr + self.mv_stage2 + self.mv_final


class _Rand:
    """Random replacement vectors from the counter-based stream."""

    def __init__(self, seed):
        self.seed = seed
        self.count = 0

    def vec(self, n):
        self.count += 1
        return _rng.stream(self.seed, self.count, n)


def _project_out(t, bases):
    for Bm in bases:
        if Bm is not None and Bm.shape[1]:
            t = t - Bm @ (Bm.T @ t)
    return t


def orth_block(T, bases, rnd: _Rand):
    """Orthonormal columns spanning T orthogonalised against ``bases``.

    Column by column: two Gram-Schmidt passes against the bases and the
    columns accepted so far (a third pass if the second still removed more
    than half).  A column whose norm drops by more than 1/DEP_DROP is
    replaced by a random vector, which is orthogonalised the same way."""
    T = np.asarray(T, dtype=np.float64)
    if T.ndim == 1:
        T = T[:, None]
    out = []
    for j in range(T.shape[1]):
        t = T[:, j].copy()
        for attempt in range(3):
            n0 = np.linalg.norm(t)
            cur = bases + ([np.column_stack(out)] if out else [])
            t1 = _project_out(t, cur)
            n1 = np.linalg.norm(t1)
            t2 = _project_out(t1, cur)
            n2 = np.linalg.norm(t2)
            if n2 < 0.5 * n1:
                t2 = _project_out(t2, cur)
                n2 = np.linalg.norm(t2)
            if n0 > 0 and n2 > DEP_DROP * n0:
                out.append(t2 / n2)
                break
            t = rnd.vec(T.shape[0])
        else:
            raise RuntimeError("could not extend the basis")
    if not out:
        return np.zeros((T.shape[0], 0))
    return np.column_stack(out)


def _small_orth_against(P, K):
    """Orthonormal columns of P orthogonalised against orthonormal K in the
    small coefficient space.  A dependent column is replaced by the next
    coordinate vector that is independent, so the result always has
    min(P.cols, rows - K.cols) columns."""
    rows = P.shape[0]
    want = min(P.shape[1], rows - K.shape[1])
    out = []
    unit = 0
    c = 0
    while len(out) < want:
        if c < P.shape[1]:
            t = P[:, c].copy()
            c += 1
        else:
            t = np.zeros(rows)
            t[unit] = 1.0
            unit += 1
        while True:
            n0 = np.linalg.norm(t)
            cur = [K] + ([np.column_stack(out)] if out else [])
            for _ in range(2):
                t = _project_out(t, cur)
            n2 = np.linalg.norm(t)
            if n0 > 0 and n2 > 1e-8 * n0:
                out.append(t / n2)
                break
            t = np.zeros(rows)
            t[unit] = 1.0
            unit += 1
    if not out:
        return np.zeros((rows, 0))
    return np.column_stack(out)


def _sym(H):
    return 0.5 * (H + H.T)


def _pad(Sc, rows):
    P = np.zeros((rows, Sc.shape[1]))
    P[: Sc.shape[0]] = Sc
    return P


# --------------------------------------------------------------------------
# Stage 1: block GD+k on C = A^T A
# --------------------------------------------------------------------------
def stage1_gdk(A, k, tol, b, pmax, pmin, X0, which="smallest", precond=None, anorm=None,
               max_restarts=10000, floor=10.0, eps=EPS64, seed=11, stats: Stats | None = None,
               max_iters=None, callback=None, fallback=None, fallback_window=25, sn2_init=0.0,
               c_apply=None, si_anorm=None):
    """Block GD+k on C for k extreme eigenpairs (Sections 2.2, 2.4, 3.1).

    ``precond(R, theta, X) -> T`` maps the residual block to the correction
    block (None: T = R).  ``callback(it, X, R, theta, X_lock)`` sees every
    iteration's Ritz block (used to harvest training pairs).  ``c_apply``
    replaces the product with C by the caller's operator (C itself, or C^-1
    for shift-invert; then ``si_anorm`` = ||A|| sets the test
    ||C^-1 x - mu x|| < delta sqrt(mu) / ||A||, the image of the test on C,
    since C r' = -mu r_C for r' = C^-1 x - mu x).  With a
    ``fallback`` preconditioner, ``precond`` is replaced by it for the rest
    of the run when the leading residual has not halved within a window of
    ``fallback_window`` iterations (the learned preconditioner's safeguard).  Returns (X_lock, theta_lock, V_rest, s_n^2, info)
    with theta ascending for 'smallest', descending for 'largest'."""
    stats = stats if stats is not None else Stats()
    n = A.shape[1]
    rnd = _Rand(seed)

    def Cop(X):
        stats.mv_stage1 += X.shape[1]
        if c_apply is not None:
            return c_apply(X)
        return A.T @ (A @ X)

    V = orth_block(X0, [], rnd)
    W = Cop(V)
    H = _sym(V.T @ W)
    Xl = np.zeros((n, 0))
    thl = []
    sn2 = float(anorm) ** 2 if anorm else float(sn2_init)
    prev = None
    hist = []
    L = max(100, 20 * int(math.ceil(pmax / b)))
    it = 0
    converged = False
    pc_hist = []
    last_rebuild = -(10**9)
    best = (np.zeros(0), np.zeros((n, 0)))
    stats.fallback = False
    while True:
        it += 1
        theta, S = np.linalg.eigh(H)
        if which == "largest":
            theta, S = theta[::-1], S[:, ::-1]
        sn2 = max(sn2, float(theta.max()))
        sn = math.sqrt(sn2)
        p = V.shape[1]
        nb = min(b, p)
        X = V @ S[:, :nb]
        R = W @ S[:, :nb] - X * theta[:nb]
        rn = np.linalg.norm(R, axis=0)
        if callback is not None:
            callback(it, X, R, theta[:nb], Xl)
        if fallback is not None and not stats.fallback:
            pc_hist.append(rn[0])
            Lf = fallback_window
            if len(pc_hist) >= 2 * Lf and min(pc_hist[-Lf:]) > 0.5 * min(pc_hist[-2 * Lf:-Lf]):
                precond = fallback
                stats.fallback = True
        need = k - len(thl)

        def rel_of(i):
            si = math.sqrt(max(theta[i], 0.0))
            return tol * si / si_anorm if si_anorm else tol * si * sn

        def thr_of(i):
            return max(rel_of(i), floor * eps * sn2)

        conv = [i for i in range(min(nb, need)) if rn[i] < thr_of(i)]
        stag = None
        # floor-limited stagnation acceptance for the leading target
        if not conv and need > 0 and rel_of(0) < floor * eps * sn2:
            hist.append(rn[0])
            if len(hist) > 2 * L and rn[0] < 10.0 * floor * eps * sn2:
                if min(hist[-L:]) > 0.9 * min(hist[:-L]):
                    conv.append(0)
                    stag = 0
        if conv and stag is None:
            # lock only on the explicit residual C x - theta x: the recurrence
            # W s - theta x drifts from it over restarts; on a mismatch the
            # basis products are recomputed, W = C V
            Xc = X[:, conv]
            Rt = Cop(Xc) - Xc * theta[conv]
            rt = np.linalg.norm(Rt, axis=0)
            ok = [i for q, i in enumerate(conv) if rt[q] < thr_of(i)]
            if len(ok) < len(conv):
                if it - last_rebuild > 10:
                    W = Cop(V)
                    H = _sym(V.T @ W)
                    prev = None
                    last_rebuild = it
                    continue
                # rebuilt within the last 10 iterations: the two residuals
                # differ by rounding only, so iterate on without locking
                conv = []
        if conv:
            hist = []
            pc_hist = []
            for i in conv:
                Xl = np.column_stack([Xl, X[:, i]])
                thl.append(float(theta[i]))
                stats.res_stage1.append(float(rn[i]))
            if len(thl) >= k:
                converged = True
                keep = [i for i in range(p) if i not in conv]
                V = V @ S[:, keep]
                break
            keep = [i for i in range(p) if i not in conv]
            V = V @ S[:, keep]
            W = W @ S[:, keep]
            H = np.diag(theta[keep])
            prev = None
            if V.shape[1] == 0:
                V = orth_block(np.column_stack([rnd.vec(n) for _ in range(b)]), [Xl], rnd)
                W = Cop(V)
                H = _sym(V.T @ W)
            continue
        if stats.restarts1 > max_restarts or (max_iters and it > max_iters):
            # out of budget: the pairs still missing are returned as the
            # leading Ritz vectors of the final basis (best approximations)
            nbest = min(need, p)
            best = (np.asarray(theta[:nbest], dtype=np.float64), V @ S[:, :nbest])
            break
        T = R if precond is None else precond(R, theta[:nb], X)
        if p + nb > pmax:
            Y = S[:, :pmin]
            if prev is not None:
                Pq = _small_orth_against(_pad(prev, p), Y)
                Y = np.column_stack([Y, Pq])
            V = V @ Y
            W = W @ Y
            H = _sym(Y.T @ H @ Y)
            prev = Y.T @ S[:, :nb]
            stats.restarts1 += 1
        else:
            prev = S[:, :nb]
        T = orth_block(T, [Xl, V], rnd)
        WT = Cop(T)
        p = V.shape[1]
        Hb = V.T @ WT
        Ht = _sym(T.T @ WT)
        H = np.block([[H, Hb], [Hb.T, Ht]])
        V = np.column_stack([V, T])
        W = np.column_stack([W, WT])
        prev = _pad(prev, V.shape[1])
    stats.iters1 += it
    order = np.argsort(thl) if which == "smallest" else np.argsort(thl)[::-1]
    thl = np.asarray(thl)[order]
    Xl = Xl[:, order]
    return Xl, thl, V, sn2, {"converged": converged, "iters": it, "best": best}


# --------------------------------------------------------------------------
# Transition: post-processing Rayleigh-Ritz (Section 3.1, Algorithm 1 step 3)
# --------------------------------------------------------------------------
def transition_rr(A, Xl, Vrest, k, pmin, anorm, seed=13, stats: Stats | None = None):
    """Rayleigh-Ritz of C on Z = orth([X_lock, leading restart vectors]).

    Returns shifts sigma (ascending), right vectors v (n x k) and left
    vectors u = A v / ||A v|| (m x k); u is random (orthogonalised against
    the other u) when ||A v|| <= 10 eps ||A|| (Section 3.3)."""
    stats = stats if stats is not None else Stats()
    rnd = _Rand(seed)
    extra = max(0, pmin - k)
    Z0 = np.column_stack([Xl, Vrest[:, :extra]]) if extra and Vrest.shape[1] else Xl
    Z = orth_block(Z0, [], rnd)
    AZ = A @ Z
    stats.mv_rr += Z.shape[1]
    Ua, s, Vt = np.linalg.svd(AZ, full_matrices=False)
    idx = np.argsort(s, kind="stable")[:k]
    sig = s[idx]
    v = Z @ Vt.T[:, idx]
    u = Ua[:, idx].copy()
    return sig, v, _random_tiny_left(u, sig, anorm, rnd)


def _random_tiny_left(u, sig, anorm, rnd):
    """Section 3.3: a left vector of a singular value <= 10 eps ||A|| carries
    no accuracy from stage 1 and is replaced by a random one, orthogonalised
    against the other left vectors."""
    k = u.shape[1]
    for i in range(k):
        if sig[i] <= 10 * EPS64 * anorm:
            others = [u[:, [j for j in range(k) if j != i and sig[j] > 10 * EPS64 * anorm]]]
            r = orth_block(rnd.vec(u.shape[0])[:, None], others, rnd)
            u[:, i] = r[:, 0]
    return u


def resume_seeds(A, V, shifts, anorm, seed=13, stats: Stats | None = None):
    """Stage-2 seeds from saved first-stage output (Algorithm 2 step 1):
    v_i the given vectors normalised, u_i = A v_i / ||A v_i||, random where
    shifts_i <= 10 eps ||A||."""
    stats = stats if stats is not None else Stats()
    v = np.asarray(V, dtype=np.float64) / np.linalg.norm(V, axis=0)
    Av = A @ v
    stats.mv_rr += v.shape[1]
    u = Av / np.where(np.linalg.norm(Av, axis=0) > 0, np.linalg.norm(Av, axis=0), 1.0)
    return v, _random_tiny_left(u, np.asarray(shifts, dtype=np.float64), anorm, _Rand(seed))


# --------------------------------------------------------------------------
# Stage 2: GD+k with refined projection on B (Algorithm 2)
# --------------------------------------------------------------------------
def _triplet_residual(x, bx, theta, n):
    """sqrt(||A^T u - theta v||^2 + ||A v - theta u||^2) for the normalised
    halves v = x_top / ||x_top||, u = x_bot / ||x_bot|| of x, from x and
    B x = [A^T x_bot; A x_top] (the stopping test of Section 5).  For a
    balanced unit x it equals sqrt(2) ||B x - theta x||; an unbalanced x
    (one half nearly zero) can pass the B test while its triplet fails."""
    nv = float(np.linalg.norm(x[:n]))
    nu = float(np.linalg.norm(x[n:]))
    if not (nv > 0.0 and nu > 0.0):
        return math.inf
    ru = bx[:n] / nu - theta * x[:n] / nv
    rv = bx[n:] / nv - theta * x[n:] / nu
    return math.sqrt(float(ru @ ru) + float(rv @ rv))


def stage2_refined(A, shifts, v0, u0, tol, anorm, b, pmax, pmin, precondB=None,
                   max_restarts=10000, seed=17, stats: Stats | None = None, max_iters=None,
                   method="gdk", max_inner=50, trace=None, best=None, extract="refined"):
    """Interior eigenpairs of B near the given shifts (Algorithm 2).

    ``method`` 'gdk' takes the (preconditioned) residual block as the
    correction (GD+k); 'jdqmr' solves the projected correction equation of
    the target, P (B - s I) P t = -r with s its shift and P the projector
    orthogonal to [locked vectors, x], by symmetric QMR with dynamic stopping
    (oracle.jdqmr; ``precondB`` then preconditions the inner solver) and
    expands by that one direction.  Inner products with B count as stage-2
    products.  ``trace``, if a list, receives (iteration, basis size, theta,
    ||r||, sigma_min(R), shift) per iteration.  ``best``, if a list, receives
    on a spent budget the approximations of the targets not locked: the
    current refined vector of the target, then the seeds of the others.

    ``extract`` 'refined' is Algorithm 2's refined projection at the
    target's shift.  'harmonic0' is for approximations without accurate
    shifts (the dynamic switching runs of Section 4.1, where the paper notes
    that only accurate shifts make a harmonic procedure unnecessary):
    harmonic Ritz pairs for the target 0, W^T W y = mu^-1 ... i.e. the pencil
    (V^T B V, (BV)^T (BV)) with W^T W = R^T R from the QR of W, taken in
    descending mu = 1 / theta_harm; the target is the first candidate with
    mu > 0 and balanced halves (|2 ||x_top||^2 - 1| < 0.1), which excludes
    the null vectors [0; w] of B that m > n brings; the shifts then only
    order the seeds.

    Returns (sigma, X) with X = [v; u] unit vectors of B, in target order;
    len(sigma) < len(shifts) when the budget ran out first."""
    stats = stats if stats is not None else Stats()
    m, n = A.shape
    N = m + n
    k2 = len(shifts)
    rnd = _Rand(seed)

    def Bop(X):
        stats.mv_stage2 += X.shape[1]
        return np.vstack([A.T @ X[n:], A @ X[:n]])

    Y0 = np.vstack([v0, u0]) / math.sqrt(2.0)
    # step 2: K_{s-k}(B, y_1) by Lanczos (full reorthogonalisation) plus the seeds
    nk = max(0, pmin - k2)
    Kb = orth_block(Y0[:, :1], [], rnd)
    t = None
    for i in range(nk):
        w = Bop(Kb[:, -1:])
        if i < nk - 1:
            Kb = np.column_stack([Kb, orth_block(w, [Kb], rnd)])
        else:
            t = w
    # at most p_min seeds in the first basis; the others enter as their
    # targets come up (re-insertion after a lock)
    Ys0 = Y0[:, :min(k2, pmin)]
    V = orth_block(np.column_stack([Ys0, Kb[:, 1:]]) if Kb.shape[1] > 1 else Ys0, [], rnd)
    W = Bop(V)
    H = _sym(V.T @ W)
    Xl = np.zeros((N, 0))
    thl = []
    j = 0
    shift = float(shifts[0])
    pend = t
    prev = None
    it = 0
    thr = tol * anorm / math.sqrt(2.0)
    last_rebuild = -(10**9)
    while True:
        if pend is not None:
            T = orth_block(pend, [Xl, V], rnd)
            WT = Bop(T)
            Hb = V.T @ WT
            H = np.block([[H, Hb], [Hb.T, _sym(T.T @ WT)]])
            V = np.column_stack([V, T])
            W = np.column_stack([W, WT])
            if prev is not None:
                prev = _pad(prev, V.shape[1])
            pend = None
        it += 1
        p = V.shape[1]
        if extract == "harmonic0":
            Ys, smin = _harmonic0(V, W, H, n)
        else:
            # R factor of W - shift V (steps 5-7; the incremental update gives
            # the same R up to column signs), then its SVD (step 9)
            Rf = np.linalg.qr(W - shift * V, mode="r")
            _, sv, Yt = np.linalg.svd(Rf)
            order = np.argsort(sv, kind="stable")
            Ys = Yt.T[:, order]
            smin = float(sv[order[0]])
        y = Ys[:, 0]
        theta = float(y @ H @ y)
        x = V @ y
        wy = W @ y
        r = wy - theta * x
        rn = float(np.linalg.norm(r))
        if trace is not None:
            trace.append((it, p, theta, rn, smin, shift))
        lock = rn < thr and _triplet_residual(x, wy, theta, n) <= tol * anorm
        if lock:
            # confirm on the explicit product B x: the recurrence W y drifts
            # from it over restarts; on a mismatch W = B V and H are rebuilt,
            # at most once in 10 iterations (as in stage 1)
            bx = Bop(x[:, None])[:, 0]
            rx = bx - theta * x
            lock = (float(np.linalg.norm(rx)) < thr
                    and _triplet_residual(x, bx, theta, n) <= tol * anorm)
            if not lock and it - last_rebuild > 10:
                W = Bop(V)
                H = _sym(V.T @ W)
                prev = None
                last_rebuild = it
                continue
        if lock:
            Xl = np.column_stack([Xl, x])
            thl.append(theta)
            j += 1
            if j >= k2:
                break
            rest = Ys[:, 1:]
            if extract == "harmonic0":
                # the harmonic vectors are not orthonormal: an orthonormal
                # basis of the complement of y, in the candidates' order
                rest = np.linalg.qr(Ys)[0][:, 1:]
            V = V @ rest
            W = W @ rest
            H = _sym(rest.T @ H @ rest)
            shift = float(shifts[j])
            pend = Y0[:, j:j + 1]
            prev = None
            continue
        if stats.restarts2 > max_restarts or (max_iters and it > max_iters):
            if best is not None:
                best.append((theta, x.copy()))
                for jj in range(j + 1, k2):
                    best.append((float(shifts[jj]), Y0[:, jj].copy()))
            break
        slots = [0]
        thetas = [theta]
        for c in range(1, p):
            if len(slots) >= b or c > 2 * b or method == "jdqmr":
                break
            if extract == "harmonic0":
                # candidates come ordered, balanced ones first
                yc = Ys[:, c] / np.linalg.norm(Ys[:, c])
                xc = V @ yc
                if abs(2.0 * float(xc[:n] @ xc[:n]) - 1.0) < 0.1:
                    slots.append(c)
                    thetas.append(float(yc @ H @ yc))
                continue
            yc = Ys[:, c]
            thc = float(yc @ H @ yc)
            xc = V @ yc
            vn2 = float(xc[:n] @ xc[:n])
            if thc > 0.5 * shift and abs(2.0 * vn2 - 1.0) < 0.1:
                slots.append(c)
                thetas.append(thc)
        Ysl = Ys[:, slots]
        X = V @ Ysl
        Rr = W @ Ysl - X * np.asarray(thetas)[None, :]
        nb = len(slots)
        if method == "jdqmr":
            def Bvec(w):
                stats.mv_stage2 += 1
                return np.concatenate([A.T @ w[n:], A @ w[:n]])

            pc = None if precondB is None else (
                lambda g: precondB(g[:, None], np.array([shift]), None)[:, 0])
            t, steps, _ = _jd.jd_correction(Bvec, x, r, theta, shift, np.column_stack([Xl, x]),
                                           thr, pc, max_inner)
            stats.inner2 += steps
            T = t[:, None]
        else:
            T = Rr if precondB is None else precondB(Rr, np.asarray(thetas), X)
        if p + nb > pmax:
            Yr = Ys[:, :pmin]
            if extract == "harmonic0":
                Yr = np.linalg.qr(Yr)[0]
            if prev is not None:
                Yr = np.column_stack([Yr, _small_orth_against(prev, Yr)])
            V = V @ Yr
            W = W @ Yr
            H = _sym(Yr.T @ H @ Yr)
            prev = Yr.T @ Ysl
            stats.restarts2 += 1
        else:
            prev = Ysl
        pend = T
    stats.iters2 += it
    return np.asarray(thl), Xl


def _harmonic0(V, W, H, n):
    """Harmonic Ritz vectors of B for the target 0 over span(V): with
    W = B V = Q R, the pairs of H y = mu R^T R y, i.e. the eigenpairs
    (mu, z) of R^-T H R^-1 with y = R^-1 z; mu = 1 / theta_harm.  Returns
    the coefficient vectors (unit columns) ordered by: balanced with mu > 0
    first, by descending mu, then the rest by descending mu; and the
    leading 1 / mu."""
    import scipy.linalg as sla

    p = V.shape[1]
    R = np.linalg.qr(W, mode="r")
    # a nearly singular R (B V rank-deficient) is regularised: diagonal
    # entries below 1e-14 max|R_jj| are raised to that size, sign kept
    d = np.diag(R).copy()
    fl = 1e-14 * np.max(np.abs(d))
    small = np.abs(d) < fl
    d[small] = np.where(d[small] < 0, -fl, fl)
    R = np.triu(R, 1) + np.diag(d)
    Ri = sla.solve_triangular(R, np.eye(p))
    mu, Z = np.linalg.eigh(_sym(Ri.T @ H @ Ri))
    Y = Ri @ Z
    Y = Y / np.linalg.norm(Y, axis=0)
    X = V @ Y
    bal = np.abs(2.0 * np.einsum("ij,ij->j", X[:n], X[:n]) - 1.0) < 0.1
    good = bal & (mu > 0)
    order = sorted(range(p), key=lambda i: (0 if good[i] else 1, -mu[i]))
    lead = mu[order[0]]
    return Y[:, order], (1.0 / lead if lead != 0 else math.inf)


# --------------------------------------------------------------------------
# Preconditioners (Section 4; Jacobi is the plain comparison arm)
# --------------------------------------------------------------------------
def jacobi_diag(A):
    """diag(C)_j = ||A_:,j||^2."""
    A2 = A.multiply(A)
    return np.asarray(A2.sum(axis=0)).ravel()


def jacobi_precond_C(d, olsen=True, clamp=1e-3):
    """t = M r with M = (diag(C) - theta I)^-1, optionally in the Olsen form
    t = M r - e M x, e = x^T M r / x^T M x (GD_Olsen_PlusK, Section 5)."""

    def apply(R, theta, X):
        T = np.empty_like(R)
        for i in range(R.shape[1]):
            den = d - theta[i]
            den = np.where(np.abs(den) < clamp * d, np.where(den >= 0, clamp * d, -clamp * d), den)
            Mr = R[:, i] / den
            if olsen:
                Mx = X[:, i] / den
                e = (X[:, i] @ Mr) / (X[:, i] @ Mx)
                Mr = Mr - e * Mx
            T[:, i] = Mr
        return T

    return apply


def jacobi_precond_B(A, d, stats: Stats):
    """B-form of a C preconditioner M = diag(C)^-1 (Section 4):
    [f; g] -> [M (A^T g); A (M f)]."""
    m, n = A.shape

    def apply(R, theta, X):
        f, g = R[:n], R[n:]
        stats.mv_prec += R.shape[1]
        return np.vstack([(A.T @ g) / d[:, None], A @ (f / d[:, None])])

    return apply


# --------------------------------------------------------------------------
# Driver
# --------------------------------------------------------------------------
def _final(A, V, U, stats, AV=None):
    """Explicit triplet residuals in float64 (Section 5 stopping test)."""
    if AV is None:
        AV = A @ V
        stats.mv_final += V.shape[1]
    sigma = np.einsum("ij,ij->j", U, AV)
    neg = sigma < 0
    U[:, neg] *= -1.0
    sigma = np.abs(sigma)
    rv = AV - U * sigma
    ru = A.T @ U - V * sigma
    res = np.sqrt((rv * rv).sum(0) + (ru * ru).sum(0))
    return sigma, res, U


def phsvds(A, k, tol=1e-12, which="smallest", block=1, precond="none", X0=None, anorm=None,
           stage2="auto", max_basis=None, min_restart=None, max_restarts=10000, floor=10.0,
           seed=2, max_iters=None, gnn_params=None, stage2_method="jdqmr", max_inner=50,
           init_V=None, shifts=None, stage2_extract="refined", c_apply=None, c_inverse=False):
    """k smallest (or largest) singular triplets of A by PHSVDS.

    Returns dict(sigma, U, V, res, stats, stage1_sigma, converged, anorm).
    ``precond`` is 'none', 'jacobi' (stage 1: Olsen-Jacobi on C; stage 2: its
    B-form) or 'gnn' (stage 1: the learned network of oracle.precond with
    gnn_params).  ``stage2_method`` is 'gdk' (GD+k with the refined
    projection) or 'jdqmr' (the same outer iteration with the correction
    equation solved by symmetric QMR, Section 3.2).  ``converged`` holds
    only if every pair locked in its last stage and every final residual
    sqrt(||r_u||^2 + ||r_v||^2) is at most tol ||A|| (Section 5).

    ``precond`` may be ("inverse_A", Minv, MinvT) for a preconditioner
    M ~ A given by its solves Minv(Y) = M^-1 Y (m rows -> n rows) and
    MinvT(X) = M^-T X (n -> m): stage 1 takes M^-1 M^-T R, stage 2
    [f; g] -> [M^-1 g; M^-T f] (Section 4, approx_A_forms).
    ``precond`` may be ("B", MB) for a preconditioner of B alone,
    MB(R, theta) -> T on (m + n) x b blocks with theta the b estimates of
    sigma (Section 4: a preconditioner directly for B); stage 1 then runs
    without one.
    ``precond`` may also be a callable M(R, theta) -> T, a preconditioner of
    C applied to an n x b block (theta: the b eigenvalue estimates of C):
    stage 1 takes T = M(R), stage 2 its B-form [M(A^T g); A M(f)] with theta
    the squared stage-2 estimates.  ``init_V`` (n x k0) without ``shifts``
    is the first stage's starting basis; with ``shifts`` it is saved
    first-stage output and the solve resumes at the second stage for all k
    pairs (left vectors from resume_seeds); ``stage2_extract`` then picks
    the second stage's extraction ('refined' at the shifts, or 'harmonic0'
    for estimates too rough to serve as shifts, see stage2_refined).

    ``c_apply(X)`` replaces the first stage's products with C by the
    caller's operator: C itself, or with ``c_inverse`` C^-1 (shift-invert,
    Section 4: the largest eigenvalues mu of C^-1 give sigma = mu^-1/2);
    the transition, the second stage and the final check still use A.  In
    shift-invert mode ||A|| is the given anorm or twelve power steps on C."""
    import workloads  # seeded inputs only

    m, n = A.shape
    if m < n:
        raise ValueError("A must have m >= n")
    stats = Stats()
    b = block
    pmax, pmin = basis_sizes(k, b, max_basis, min_restart, n)
    if X0 is None:
        X0 = workloads.initial_block(n, b, seed)
    pc1 = pcB = fb = None
    if isinstance(precond, tuple) and precond[0] == "inverse_A":
        pc1, pcB = approx_A_forms(precond[1], precond[2], n)
    elif isinstance(precond, tuple) and precond[0] == "B":
        fB = precond[1]

        def pcB(R, theta, X):
            return fB(R, np.asarray(theta))
    elif callable(precond):
        M = precond

        def pc1(R, theta, X):
            return M(R, np.asarray(theta))

        def pcB(R, theta, X):
            th2 = np.asarray(theta) ** 2
            f, g = R[:n], R[n:]
            stats.mv_prec += R.shape[1]
            return np.vstack([M(A.T @ g, th2), A @ M(f, th2)])
    elif precond == "jacobi":
        d = jacobi_diag(A)
        pc1 = jacobi_precond_C(d)
        pcB = jacobi_precond_B(A, d, stats)
    elif precond == "gnn":
        from . import precond as pcmod
        g = pcmod.Graph(A)
        d = jacobi_diag(A)
        fb = jacobi_precond_C(d)

        def pc1(R, theta, X):
            return np.column_stack([pcmod.forward(g, gnn_params, R[:, i], X[:, i], theta[i])[0]
                                    for i in range(R.shape[1])])
    elif precond != "none":
        raise ValueError(precond)
    if init_V is not None and shifts is not None:
        # resume at the second stage from saved first-stage output
        an = float(anorm) if anorm else math.sqrt(_power_norm2(A, seed, stats))
        order = np.argsort(np.asarray(shifts[:k]), kind="stable")
        sh = np.asarray(shifts[:k], dtype=np.float64)[order]
        v0, u0 = resume_seeds(A, np.asarray(init_V)[:, :k][:, order], sh, an, stats=stats)
        stats.stage2_pairs = k
        th2, X2 = stage2_refined(A, sh, v0, u0, tol, an, b, pmax, pmin, pcB, max_restarts,
                                 stats=stats, max_iters=max_iters, method=stage2_method,
                                 max_inner=max_inner, extract=stage2_extract)
        got = X2.shape[1]
        V = np.column_stack([X2[:n], v0[:, got:]])
        U = np.column_stack([X2[n:], u0[:, got:]])
        V = V / np.linalg.norm(V, axis=0)
        U = U / np.linalg.norm(U, axis=0)
        sigma, res, U = _final(A, V, U, stats)
        o2 = np.argsort(sigma, kind="stable")
        sigma, res, U, V = sigma[o2], res[o2], U[:, o2], V[:, o2]
        for i in range(V.shape[1]):
            if V[np.argmax(np.abs(V[:, i])), i] < 0:
                V[:, i] *= -1.0
                U[:, i] *= -1.0
        stats.anorm_est = an
        converged = got == k and bool(np.all(res <= tol * an * (1.0 + 1e-8)))
        return {"sigma": sigma, "U": U, "V": V, "res": res, "stats": stats,
                "stage1_sigma": sh, "converged": converged, "anorm": an}
    if init_V is not None:
        X0 = np.asarray(init_V, dtype=np.float64)
    sn2_init = 0.0
    if precond == "gnn" and not anorm:
        # the learned preconditioner smooths, so the basis does not reach
        # the top of the spectrum: start the ||A||^2 estimate from twelve
        # steps of power iteration on C (a lower bound)
        sn2_init = _power_norm2(A, seed, stats)
    if c_inverse:
        if c_apply is None or which != "smallest" or pc1 is not None:
            raise ValueError("shift-invert needs c_apply, the smallest end and no preconditioner")
        sn2 = float(anorm) ** 2 if anorm else _power_norm2(A, seed, stats)
        Xl, thl, Vr, _, info = stage1_gdk(A, k, tol, b, pmax, pmin, X0, "largest", None, None,
                                          max_restarts, floor, EPS64, stats=stats,
                                          max_iters=max_iters, c_apply=c_apply,
                                          si_anorm=math.sqrt(sn2))
        # eigenvalues mu of C^-1 -> theta = 1 / mu of C, ascending
        thl = 1.0 / np.asarray(thl)[::-1]
        Xl = Xl[:, ::-1]
        bth, bX = info["best"]
        info["best"] = (1.0 / bth if bth.size else bth, bX)
    else:
        Xl, thl, Vr, sn2, info = stage1_gdk(A, k, tol, b, pmax, pmin, X0, which, pc1, anorm,
                                            max_restarts, floor, EPS64, stats=stats,
                                            max_iters=max_iters,
                                            fallback=fb if precond == "gnn" else None,
                                            sn2_init=sn2_init, c_apply=c_apply)
    sn = math.sqrt(sn2)
    stats.anorm_est = sn
    an = float(anorm) if anorm else sn
    s1 = np.sqrt(np.maximum(thl, 0.0))
    kk = len(thl)
    if which == "largest" or stage2 == "never":
        need2 = 0
    elif stage2 == "force":
        need2 = kk
    else:
        need2 = int(np.sum(tol * s1 < floor * EPS64 * sn))
    locked2 = need2
    Xbest = info["best"][1]
    if need2 == 0:
        V = np.column_stack([Xl, Xbest])
        AV = A @ V
        stats.mv_final += V.shape[1]
        nv = np.linalg.norm(AV, axis=0)
        U = AV / np.where(nv > 0, nv, 1.0)
        sigma, res, U = _final(A, V, U, stats, AV)
    else:
        sig_rr, v_rr, u_rr = transition_rr(A, Xl, Vr, kk, pmin, an, stats=stats)
        stats.stage2_pairs = need2
        th2, X2 = stage2_refined(A, sig_rr[:need2], v_rr[:, :need2], u_rr[:, :need2], tol, an,
                                 b, pmax, pmin, pcB, max_restarts, stats=stats,
                                 max_iters=max_iters, method=stage2_method, max_inner=max_inner)
        got = X2.shape[1]
        locked2 = got
        Ub = A @ Xbest
        stats.mv_rr += Xbest.shape[1]
        V = np.column_stack([X2[:n], v_rr[:, got:], Xbest])
        U = np.column_stack([X2[n:], u_rr[:, got:], Ub])
        V = V / np.linalg.norm(V, axis=0)
        U = U / np.where(np.linalg.norm(U, axis=0) > 0, np.linalg.norm(U, axis=0), 1.0)
        sigma, res, U = _final(A, V, U, stats)
    order = np.argsort(sigma, kind="stable")
    if which == "largest":
        order = order[::-1]
    sigma, res, U, V = sigma[order], res[order], U[:, order], V[:, order]
    for i in range(V.shape[1]):
        jmax = np.argmax(np.abs(V[:, i]))
        if V[jmax, i] < 0:
            V[:, i] *= -1.0
            U[:, i] *= -1.0
    converged = (bool(info["converged"]) and len(sigma) == k and locked2 == need2
                 and bool(np.all(res <= tol * an * (1.0 + 1e-8))))
    return {"sigma": sigma, "U": U, "V": V, "res": res, "stats": stats,
            "stage1_sigma": s1, "converged": converged, "anorm": an}


def approx_A_forms(Minv, MinvT, n):
    """Section 4: from M ~ A (solves with M and M^T), the preconditioner of
    C = A^T A is M^-1 M^-T and that of B = [0 A^T; A 0] is
    [0 M^-1; M^-T 0], i.e. [f; g] -> [M^-1 g; M^-T f] (no product with A)."""

    def pc1(R, theta, X):
        return Minv(MinvT(R))

    def pcB(R, theta, X):
        return np.vstack([Minv(R[n:]), MinvT(R[:n])])

    return pc1, pcB


def _power_norm2(A, seed, stats):
    """||C x|| after twelve steps of power iteration on C = A^T A from a
    counter-based random start: a lower bound on ||A||^2."""
    x = _Rand(seed + 7).vec(A.shape[1])
    lam = 0.0
    for it in range(13):
        nx = float(np.linalg.norm(x))
        if not nx > 0:
            break
        if it > 0:
            lam = nx
        if it == 12:
            break
        x = A.T @ (A @ (x / nx))
        stats.mv_prec += 1
    return lam


def harvest(A, k, b, every=5, max_pairs=64, tol=1e-8, seed=2, cg_tol=1e-8, cg_maxit=2000,
            max_iters=None, shift_scale=1.0):
    """Training pairs for the learned preconditioner from a stage-1 run:
    every ``every`` iterations, each targeted Ritz pair (theta_i, x_i) with
    residual r_i gives the exact correction t* of
    (I-QQ^T)(C - rho theta_i I)(I-QQ^T) t = -r_i, t orthogonal to
    Q = [X_lock, Ritz block] (projected CG), rho = shift_scale (1: the
    Jacobi-Davidson correction equation, 0: the projected C^-1 r).  Pairs
    whose CG meets non-positive curvature or does not converge are dropped.
    Returns (r, x, theta, t*, Q) per pair.  Parity unpinned beyond the
    equation itself (which pairs are taken depends on the iteration path)."""
    import workloads
    from . import precond as pcmod
    n = A.shape[1]
    pmax, pmin = basis_sizes(k, b)
    X0 = workloads.initial_block(n, b, seed)
    out = []

    def cb(it, X, R, theta, Xl):
        if it % every or len(out) >= max_pairs:
            return
        for i in range(X.shape[1]):
            if len(out) >= max_pairs:
                return
            Q = np.column_stack([Xl, X])
            t, its, ok = pcmod.projected_cg(A, shift_scale * float(theta[i]), Q, R[:, i], cg_tol,
                                            cg_maxit)
            if ok:
                out.append((R[:, i].copy(), X[:, i].copy(), float(theta[i]), t, Q))

    stage1_gdk(A, k, tol, b, pmax, pmin, X0, callback=cb, max_iters=max_iters)
    return out
