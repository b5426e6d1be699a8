"""Pins of the learned-preconditioner oracle: finite differences of the
back-propagated gradient, invariants of the network (projection, positive
homogeneity, graph-permutation equivariance), Adam's closed-form first
step, and the projected CG against a dense solve of the projected system."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import phsvds as ph
from oracle import precond as pc


def _setup(width=8, seed=0):
    A = wl.random_sparse(60, 40, 5, seed=11)
    g = pc.Graph(A)
    P = wl.gnn_init_weights(width, seed=seed)
    r = np.random.default_rng(1)
    rv = r.standard_normal(40)
    x = r.standard_normal(40)
    x /= np.linalg.norm(x)
    rv -= x * (x @ rv)
    tstar = r.standard_normal(40)
    tstar -= x * (x @ tstar)
    return A, g, P, rv, x, 0.3, tstar


@pytest.mark.parametrize("kind", ["target", "residual"])
def test_gradient_matches_central_differences(kind):
    A, g, P, r, x, th, ts = _setup()
    # biases are zero at init: move them off zero so relu masks are generic
    rr = np.random.default_rng(5)
    for k in ("b1", "b2", "b3"):
        P[k] = 0.1 * rr.standard_normal(P[k].shape)
    loss, grads = pc.loss_and_grad(g, P, r, x, th, ts, kind)
    h = 1e-6
    for k in pc.NAMES:
        flat = P[k].ravel()
        for idx in rr.choice(flat.size, size=min(4, flat.size), replace=False):
            Pp = {kk: v.copy() for kk, v in P.items()}
            Pm = {kk: v.copy() for kk, v in P.items()}
            Pp[k].ravel()[idx] += h
            Pm[k].ravel()[idx] -= h
            lp, _ = pc.loss_and_grad(g, Pp, r, x, th, ts, kind)
            lm, _ = pc.loss_and_grad(g, Pm, r, x, th, ts, kind)
            fd = (lp - lm) / (2 * h)
            an = grads[k].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, an)


def test_output_orthogonal_to_ritz_vector_and_homogeneous():
    A, g, P, r, x, th, ts = _setup()
    t, _ = pc.forward(g, P, r, x, th)
    assert abs(t @ x) < 1e-12 * np.linalg.norm(t)
    t2, _ = pc.forward(g, P, 3.7 * r, x, th)
    assert np.allclose(t2, 3.7 * t, rtol=1e-12, atol=1e-14)


def test_graph_permutation_equivariance():
    A, g, P, r, x, th, ts = _setup()
    perm = np.random.default_rng(3).permutation(40)
    Pm = sp.csr_matrix(np.eye(40)[:, perm])  # column permutation: (A Pm)_{:, j} = A_{:, perm[j]}
    A2 = (A @ Pm).tocsr()
    g2 = pc.Graph(A2)
    t, _ = pc.forward(g, P, r, x, th)
    t2, _ = pc.forward(g2, P, r[perm], x[perm], th)
    assert np.allclose(t2, t[perm], rtol=1e-12, atol=1e-14)


def test_adam_first_steps_closed_form():
    P = {k: np.ones(v) for k, v in pc.shapes(4).items()}
    G = {k: np.full(v, -2.0) for k, v in pc.shapes(4).items()}
    m = {k: np.zeros(v) for k, v in pc.shapes(4).items()}
    v = {k: np.zeros(v) for k, v in pc.shapes(4).items()}
    P1, m1, v1 = pc.adam_step(P, G, m, v, 1, lr=0.01)
    # step 1: m_hat = g, v_hat = g^2 -> update lr * g / (|g| + eps)
    assert np.allclose(P1["wo"], 1.0 + 0.01 * 2.0 / (2.0 + 1e-8))
    G2 = {k: np.full(v, 4.0) for k, v in pc.shapes(4).items()}
    P2, _, _ = pc.adam_step(P1, G2, m1, v1, 2, lr=0.01)
    mk = 0.9 * 0.1 * -2.0 + 0.1 * 4.0
    vk = 0.999 * 0.001 * 4.0 + 0.001 * 16.0
    upd = 0.01 * (mk / (1 - 0.81)) / (math.sqrt(vk / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(P2["b3"], P1["b3"] - upd)


def test_projected_cg_matches_dense_solve():
    A = wl.random_sparse(80, 50, 6, seed=4)
    C = (A.T @ A).toarray()
    lam, Vx = np.linalg.eigh(C)
    theta = 0.5 * (lam[0] + lam[1])
    x = Vx[:, 0] + 1e-3 * np.random.default_rng(0).standard_normal(50)
    x /= np.linalg.norm(x)
    Q = x[:, None]
    r = C @ x - (x @ C @ x) * x
    t, its, ok = pc.projected_cg(A, theta, Q, r, tol=1e-12, maxit=500)
    assert ok
    Z = np.linalg.qr(np.column_stack([Q, np.eye(50)]))[0][:, 1:50]
    y = np.linalg.solve(Z.T @ (C - theta * np.eye(50)) @ Z, -Z.T @ r)
    assert np.allclose(t, Z @ y, rtol=1e-8, atol=1e-10 * np.linalg.norm(t))
    assert abs(x @ t) < 1e-12 * np.linalg.norm(t)


@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_harvest_pairs_solve_their_correction_equation(rho):
    """(I-QQ^T)((C - rho theta I) t + r) = 0 and Q^T t = 0 for every pair."""
    A = wl.random_sparse(300, 200, 8, seed=2000)
    pairs = ph.harvest(A, 4, 2, every=3, max_pairs=6, max_iters=30, shift_scale=rho)
    assert len(pairs) >= 3
    for r, x, th, t, Q in pairs:
        v = (A.T @ (A @ t) - rho * th * t) + r
        v -= Q @ (Q.T @ v)
        assert np.max(np.abs(Q.T @ t)) < 1e-10 * np.linalg.norm(t)
        assert np.linalg.norm(v) < 1e-6 * np.linalg.norm(r)


def test_gnn_preconditioned_oracle_converges_with_fallback():
    """An untrained network is no preconditioner; the safeguard switches to
    Jacobi and the method still converges to the definition's triplets."""
    A = wl.random_sparse(300, 200, 8, seed=2001)
    sig = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:3]
    an = np.linalg.norm(A.toarray(), 2)
    out = ph.phsvds(A, 3, 1e-12, block=2, anorm=an, precond="gnn",
                    gnn_params=wl.gnn_init_weights(8, seed=1))
    assert out["converged"]
    assert np.allclose(out["sigma"], sig, rtol=1e-10)
    assert np.all(out["res"] <= 1e-12 * an)


def test_polynomial_weights_give_the_symmetric_polynomial_preconditioner():
    """With the polynomial weights of workloads.gnn_poly_weights and theta = 0
    the network is, by construction, the operator
    t = (I - x x^T) D^-1/2 p(Ch) D^-1/2 r / mean(diag C) with Ch =
    D^-1/2 A^T A D^-1/2 (D = diag C / mean diag C); checked against that
    closed form built from dense matrices (width 8 and 32, degree 1 to 3)."""
    A = wl.random_sparse(300, 200, 6, seed=9)
    Cd = (A.T @ A).toarray()
    dC = np.diag(Cd).copy()
    dm = dC.mean()
    Dn = dC / dm
    Chd = Cd / np.sqrt(np.outer(dC, dC))
    g = pc.Graph(A)
    r = np.random.default_rng(1).standard_normal(200)
    x = np.random.default_rng(2).standard_normal(200)
    x /= np.linalg.norm(x)
    for width in (8, 32):
        for coeffs in ([0.7], [2.0, -0.5], [3.0, -2.5, 0.6], [3.67, -3.94, 1.61, -0.22]):
            P = wl.gnn_poly_weights(coeffs, width)
            t, _ = pc.forward(g, P, r, x, 0.0)
            pC = sum(c * np.linalg.matrix_power(Chd, k) for k, c in enumerate(coeffs))
            ref = (pC @ (r / np.sqrt(Dn))) / np.sqrt(Dn) / dm
            ref -= x * (x @ ref)
            assert np.allclose(t, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_inverse_poly_coeffs_fit():
    """x p(x) approximates 1 on (0, hi]: the fit error falls with the degree
    and p is positive on the interval for degree 3."""
    errs = []
    xs = np.linspace(0.01, 3.0, 500)
    for deg in (1, 2, 3):
        c = wl.inverse_poly_coeffs(3.0, deg)
        p = np.polyval(c[::-1], xs)
        errs.append(np.sqrt(np.mean((xs * p - 1) ** 2)))
    assert errs[0] > errs[1] > errs[2]
    assert np.all(np.polyval(wl.inverse_poly_coeffs(3.0, 3)[::-1], xs) > 0)


def test_residual_loss_definition():
    """The residual loss is ||A^T A t - r||^2 / ||r||^2 of the network's
    output, formed here from the dense C."""
    A, g, P, r, x, th, ts = _setup()
    t, _ = pc.forward(g, P, r, x, th)
    C = (A.T @ A).toarray()
    loss, _ = pc.loss_and_grad(g, P, r, x, th, None, "residual")
    assert loss == pytest.approx(float(np.sum((C @ t - r) ** 2) / (r @ r)), rel=1e-12)
