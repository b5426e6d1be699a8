"""Inner solver of the JDQMR second stage, float64 (test oracle).

Section 3.2 prefers an inner-outer eigensolver for the interior problem on
B = [0 A^T; A 0]: each outer step solves the Jacobi-Davidson correction
equation approximately, with the inner Krylov solver stopped dynamically.
The paper names the method (JDQMR) but defers its inner details to the
eigensolver it runs; the readings below are this project's and bind the GPU
path too.

Correction equation for the refined vector x (unit, orthogonal to the locked
vectors), its residual r = B x - theta x and the target shift eta:

    P (B - eta I) P t = -r,   t orthogonal to Q,   P = I - Q Q^T,
    Q = [locked vectors, x].

Inner solver: symmetric QMR (Freund & Nachtigal) in its form as quasi-minimal
residual smoothing of the conjugate-gradient recurrences, which stays defined
for the indefinite operator above.  With c-recurrences (theta_k, c_k, tau_k):

    CG step        q = Op w, alpha = rho / w^T q, g <- g - alpha q
    smoothing      th = ||g|| / tau, c^2 = 1 / (1 + th^2), tau <- tau th c
                   d <- c^2 th_prev^2 d + c^2 alpha w,  t <- t + d
    true residual  e <- c^2 th_prev^2 e + c^2 alpha q,  s <- s - e  (e = Op d)
    next direction z = M g, beta = g^T z / rho, w <- z + beta w

Without a preconditioner the CG residuals g are mutually orthogonal, so the
smoothed residual s has norm tau exactly (a fact the tests pin).

Eigen-residual of the outer candidate z = x + t (exact up to the locked
vectors' own residuals): with s the correction equation's residual,
(B - eta) z = -s + a x with a = theta - eta + r^T t, so for mu = eta + b
    ||(B - mu) z||^2 = ||s||^2 + 2 b s^T t + b^2 ||t||^2 + (a - b)^2,
minimised by b = (a - s^T t) / (1 + ||t||^2); the estimate is that minimum
over ||z||^2 = 1 + ||t||^2.

Dynamic stopping (this project's reading of "stops the inner linear solver
dynamically"), first that holds:
  1. the eigen-residual estimate is below the outer threshold (the new
     direction already meets the stopping test);
  2. ||s|| < 0.1 x the estimate: the linear system is solved well past what
     the current shift lets the eigen-residual gain;
  3. no 1% decrease of the estimate over the last 20 inner steps;
  4. max_inner steps.
"""
from __future__ import annotations

import math

import numpy as np

STAG_WINDOW = 20
STAG_RATIO = 0.99
LIN_RATIO = 0.1


def sqmr(op, b, prec=None, maxit=100, stop=None):
    """Symmetric QMR for op(t) = b from t = 0.

    ``op`` and ``prec`` are symmetric linear maps (prec = None: identity).
    ``stop(k, t, s, tau)`` is called after step k with the iterate, its
    residual b - op(t) (by recurrence) and the quasi-residual norm; a true
    return value ends the iteration.  Returns (t, s, steps, reason)."""
    b = np.asarray(b, dtype=np.float64)
    t = np.zeros_like(b)
    s = b.copy()
    d = np.zeros_like(b)
    e = np.zeros_like(b)
    g = b.copy()
    z = g if prec is None else prec(g)
    w = z.copy()
    rho = float(g @ z)
    tau = float(np.linalg.norm(g))
    th_prev = 0.0
    if tau == 0.0:
        return t, s, 0, "zero"
    for k in range(1, maxit + 1):
        q = op(w)
        sig = float(w @ q)
        if sig == 0.0 or rho == 0.0:
            return t, s, k - 1, "breakdown"
        alpha = rho / sig
        g = g - alpha * q
        th = float(np.linalg.norm(g)) / tau
        c2 = 1.0 / (1.0 + th * th)
        tau = tau * th * math.sqrt(c2)
        f = c2 * th_prev * th_prev
        d = f * d + (c2 * alpha) * w
        e = f * e + (c2 * alpha) * q
        t = t + d
        s = s - e
        th_prev = th
        if stop is not None:
            why = stop(k, t, s, tau)
            if why:
                return t, s, k, why
        z = g if prec is None else prec(g)
        rho_new = float(g @ z)
        w = z + (rho_new / rho) * w
        rho = rho_new
    return t, s, maxit, "max"


def eig_residual_estimate(r, theta, eta, t, s):
    """||(B - mu) z|| / ||z|| for z = x + t at the optimal mu (module notes)."""
    a = theta - eta + float(r @ t)
    tt = float(t @ t)
    st = float(s @ t)
    ss = float(s @ s)
    b = (a - st) / (1.0 + tt)
    f = ss + 2.0 * b * st + b * b * tt + (a - b) ** 2
    return math.sqrt(max(f, 0.0) / (1.0 + tt))


def jd_correction(Bop, x, r, theta, eta, Q, thr, prec=None, max_inner=50):
    """Approximate solution t of the projected correction equation (module
    notes) by sQMR with the dynamic stopping rules.  ``Bop`` maps a vector
    to B times it; ``prec`` (optional) a symmetric preconditioner, applied
    between the projections.  Returns (t, inner steps, reason)."""
    Q = np.asarray(Q, dtype=np.float64)
    if Q.ndim == 1:
        Q = Q[:, None]

    def proj(y):
        return y - Q @ (Q.T @ y)

    def op(w):
        return proj(Bop(w) - eta * w)

    pc = None if prec is None else (lambda g: proj(prec(g)))
    rhs = proj(-np.asarray(r, dtype=np.float64))
    hist = []

    def stop(k, t, s, tau):
        est = eig_residual_estimate(r, theta, eta, t, s)
        hist.append(est)
        if est < thr:
            return "converged"
        if math.sqrt(float(s @ s)) < LIN_RATIO * est:
            return "linear"
        if len(hist) > STAG_WINDOW and min(hist[-STAG_WINDOW:]) > STAG_RATIO * min(hist[:-STAG_WINDOW]):
            return "stagnation"
        return None

    t, s, steps, why = sqmr(op, rhs, pc, max_inner, stop)
    return proj(t), steps, why
