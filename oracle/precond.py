"""Learned preconditioner and exact corrections, float64 (test oracle).

The paper accepts any preconditioner for C (Section 4) and applies it as
t = Prec(r) in the correction step (Algorithm 2 step 13).  The learned one
here is a message-passing network over the sparsity graph of C = A^T A that
maps a residual r of a Ritz pair (theta, x) to an approximate correction of
(C - theta I), trained on exact corrections of the projected correction
equation

    (I - Q Q^T)(C - theta I)(I - Q Q^T) t = -r,   t orthogonal to Q,

(Q = locked vectors plus x), solved by conjugate gradients.

Network (width w, three layers):
    d_j   = C_jj / mean(diag C),  tau = theta / mean(diag C)
    rh    = r sqrt(n) / ||r||,    u = rh / sqrt(d)
    h0_j  = [u_j, u_j d_j / max(d_j - tau, d_j / 10), d_j, tau]
    h^l   = relu(h^{l-1} Ws_l + b_l + Ch (h^{l-1} Wm_l)),  l = 1..3
    Ch    = D^-1/2 A^T A D^-1/2  (applied as two sparse products)
    t~_j  = (h^3 wo + h0[:, 1])_j ||r|| / (sqrt(n) mean(diag C) sqrt(d_j))
    t     = (I - x x^T) t~
The input is scaled by D^-1/2 and the output again by D^-1/2, so that the
linear part of the network, a polynomial q in Ch, acts as the symmetric
operator D^-1/2 q(Ch) D^-1/2 (a nonsymmetric form such as q(Ch) D^-1 makes
the GD+k iteration stall); h0[:, 1] through the readout is exactly the
Jacobi step r / max(C_jj - theta, C_jj / 10), so the zero network is the
Jacobi preconditioner and the network learns a correction to it.
Loss of one sample: ||t - t*||^2 / ||t*||^2 (t* is orthogonal to x).
Optimiser: Adam (Kingma & Ba), lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8.

Parity of the trained network's quality: unpinned (measured by product counts
and time against Jacobi and no preconditioner on held-out matrices).
"""
from __future__ import annotations

import math

import numpy as np

NAMES = ["Ws1", "Wm1", "b1", "Ws2", "Wm2", "b2", "Ws3", "Wm3", "b3", "wo"]


def shapes(width=32, nin=4):
    w = width
    return {"Ws1": (nin, w), "Wm1": (nin, w), "b1": (w,), "Ws2": (w, w), "Wm2": (w, w),
            "b2": (w,), "Ws3": (w, w), "Wm3": (w, w), "b3": (w,), "wo": (w,)}


def flatten(params, width=32):
    return np.concatenate([np.asarray(params[k], dtype=np.float64).ravel() for k in NAMES])


def unflatten(vec, width=32):
    out, at = {}, 0
    for k in NAMES:
        shp = shapes(width)[k]
        size = int(np.prod(shp))
        out[k] = np.asarray(vec[at:at + size], dtype=np.float64).reshape(shp)
        at += size
    assert at == len(vec)
    return out


class Graph:
    """A, diag(C) and the symmetric normalised operator Ch = D^-1/2 A^T A D^-1/2."""

    def __init__(self, A):
        self.A = A.tocsr()
        self.At = self.A.T.tocsr()
        self.d = np.asarray(self.A.multiply(self.A).sum(axis=0)).ravel()
        self.dmean = float(self.d.mean())
        self.isd = 1.0 / np.sqrt(self.d)

    def Ch(self, Z):
        Y = self.A @ (Z * self.isd[:, None])
        return (self.At @ Y) * self.isd[:, None]


def features(g: Graph, r, theta):
    n = r.shape[0]
    nr = np.linalg.norm(r)
    rh = r * math.sqrt(n) / nr
    d = g.d / g.dmean
    tau = theta / g.dmean
    den = np.maximum(d - tau, 0.1 * d)
    u = rh / np.sqrt(d)
    return np.column_stack([u, u * d / den, d, np.full(n, tau)]), nr


def forward(g: Graph, P, r, x, theta):
    """Correction t for residual r of the Ritz pair (theta, x); also the
    intermediate values needed by the backward pass."""
    n = r.shape[0]
    h0, nr = features(g, r, theta)
    hs, pres, aggs = [h0], [], []
    h = h0
    for l in (1, 2, 3):
        M = h @ P[f"Wm{l}"]
        agg = g.Ch(M)
        pre = h @ P[f"Ws{l}"] + P[f"b{l}"][None, :] + agg
        h = np.maximum(pre, 0.0)
        pres.append(pre)
        hs.append(h)
    scale = nr / (math.sqrt(n) * g.dmean)
    osc = scale / np.sqrt(g.d / g.dmean)  # per-node output scale
    traw = (h @ P["wo"] + h0[:, 1]) * osc
    t = traw - x * (x @ traw)
    return t, {"hs": hs, "pres": pres, "scale": scale, "osc": osc}


def loss_and_grad(g: Graph, P, r, x, theta, tstar, kind="target"):
    """Loss and its gradient by back-propagation.  kind 'target':
    ||t - t*||^2 / ||t*||^2, the distance to the exact correction; kind
    'residual': ||C t - r||^2 / ||r||^2, how far t is from solving C t = r
    (tstar unused), whose gradient with respect to t is 2 C (C t - r) /
    ||r||^2."""
    t, cache = forward(g, P, r, x, theta)
    if kind == "residual":
        nr2 = float(r @ r)
        e = g.At @ (g.A @ t) - r
        loss = float(e @ e) / nr2
        gt = 2.0 * (g.At @ (g.A @ e)) / nr2
    else:
        nt = float(tstar @ tstar)
        diff = t - tstar
        loss = float(diff @ diff) / nt
        gt = 2.0 * diff / nt
    graw = gt - x * (x @ gt)  # through the projection (I - x x^T)
    hs, pres, osc = cache["hs"], cache["pres"], cache["osc"]
    grads = {}
    go = graw * osc
    grads["wo"] = hs[3].T @ go
    dh = np.outer(go, P["wo"])
    for l in (3, 2, 1):
        delta = dh * (pres[l - 1] > 0)
        hin = hs[l - 1]
        grads[f"Ws{l}"] = hin.T @ delta
        grads[f"b{l}"] = delta.sum(axis=0)
        dM = g.Ch(delta)  # Ch is symmetric
        grads[f"Wm{l}"] = hin.T @ dM
        dh = delta @ P[f"Ws{l}"].T + dM @ P[f"Wm{l}"].T
    return loss, grads


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new params, m, v."""
    out_p, out_m, out_v = {}, {}, {}
    for k in NAMES:
        mk = b1 * m[k] + (1 - b1) * grads[k]
        vk = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = mk / (1 - b1 ** step)
        vh = vk / (1 - b2 ** step)
        out_p[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
        out_m[k], out_v[k] = mk, vk
    return out_p, out_m, out_v


def projected_cg(A, theta, Q, r, tol=1e-8, maxit=2000):
    """t orthogonal to Q with (I-QQ^T)(C - theta I)(I-QQ^T) t = -(I-QQ^T) r,
    by conjugate gradients (the operator is SPD on the complement of Q when
    theta is below the spectrum left there).  Returns (t, iterations, ok);
    ok is False on non-positive curvature or no convergence."""
    Q = np.asarray(Q, dtype=np.float64)

    def proj(v):
        return v - Q @ (Q.T @ v)

    def op(v):
        v = proj(v)
        return proj(A.T @ (A @ v) - theta * v)

    b = -proj(r)
    t = np.zeros_like(b)
    res = b.copy()
    p = res.copy()
    rr = float(res @ res)
    nb = math.sqrt(rr)
    if nb == 0:
        return t, 0, True
    for it in range(1, maxit + 1):
        Ap = op(p)
        pAp = float(p @ Ap)
        if pAp <= 0:
            return proj(t), it, False
        alpha = rr / pAp
        t = t + alpha * p
        res = res - alpha * Ap
        rr_new = float(res @ res)
        if math.sqrt(rr_new) <= tol * nb:
            return proj(t), it, True
        p = res + (rr_new / rr) * p
        rr = rr_new
    return proj(t), maxit, False
