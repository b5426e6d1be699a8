"""Learned preconditioner on the GPU (float32) vs the float64 oracle:
forward output (every entry within 1e-5 of the largest), back-propagated
gradient (every entry within 1e-3 of its tensor's largest),
Adam step; harvested pairs satisfy their correction equation; the
preconditioned solver still returns the definition's triplets."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import precond as pc
from tests.gpu_util import as_np, gpu, need_gpu, say, to_dev


def _case(width=32, seed=0):
    A = wl.random_sparse(600, 400, 8, seed=31)
    P = wl.gnn_init_weights(width, seed=seed)
    rr = np.random.default_rng(seed + 5)
    for k in ("b1", "b2", "b3"):
        P[k] = (0.1 * rr.standard_normal(P[k].shape)).astype(np.float32).astype(np.float64)
    x = rr.standard_normal(400)
    x /= np.linalg.norm(x)
    r = rr.standard_normal(400)
    r -= x * (x @ r)
    ts = rr.standard_normal(400)
    ts -= x * (x @ ts)
    # float32-representable inputs so both sides see the same data
    f = lambda v: v.astype(np.float32).astype(np.float64)
    return A, P, f(r), f(x), 0.37, f(ts)


def _dev32(v):
    return torch.tensor(v, dtype=torch.float32, device="cuda")


@gpu
@pytest.mark.parametrize("width", [8, 32])
def test_gnn_forward_matches_oracle(width):
    need_gpu()
    import paper_1408_5535_amd as P
    A, Pw, r, x, th, ts = _case(width)
    say("gnn forward width", width)
    g = P.GnnGraph(to_dev(A), width)
    t = as_np(g.forward(P.gnn_pack(Pw), _dev32(r), _dev32(x), th)).astype(np.float64)
    tref, _ = pc.forward(pc.Graph(A), Pw, r, x, th)
    # element by element, against the largest entry (float32 kernels vs the
    # float64 oracle through three layers)
    err = np.max(np.abs(t - tref)) / np.max(np.abs(tref))
    say("max elementwise error / max |t|", err)
    assert err < 1e-5


@gpu
@pytest.mark.parametrize("kind", ["target", "residual"])
def test_gnn_gradient_matches_oracle(kind):
    need_gpu()
    import paper_1408_5535_amd as P
    A, Pw, r, x, th, ts = _case(32)
    say("gnn gradient width 32, loss", kind)
    g = P.GnnGraph(to_dev(A), 32)
    nw = P.gnn_nweights(32)
    grad = torch.zeros(nw, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    g.loss_grad(P.gnn_pack(Pw), _dev32(r), _dev32(x), th, _dev32(ts), grad, loss, kind)
    lref, gref = pc.loss_and_grad(pc.Graph(A), Pw, r, x, th, ts, kind)
    assert abs(loss.item() - lref) <= 1e-4 * lref
    gg = P.gnn_unpack(grad, 32)
    for k in pc.NAMES:
        # every entry of every weight tensor, against the tensor's largest
        scale = max(np.max(np.abs(gref[k])), 1e-30)
        err = np.max(np.abs(gg[k] - gref[k])) / scale
        say(k, err)
        assert err <= 1e-3, (k, err)


@gpu
def test_gnn_adam_matches_oracle():
    need_gpu()
    import paper_1408_5535_amd as P
    Pw = wl.gnn_init_weights(8, seed=3)
    G = {k: np.random.default_rng(i).standard_normal(v.shape) for i, (k, v) in enumerate(Pw.items())}
    w = P.gnn_pack(Pw)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    gflat = torch.tensor(np.concatenate([G[k].ravel() for k in P.GNN_NAMES]), device="cuda")
    P.gnn_adam(w, m, v, gflat, 1, lr=1e-2)
    zeros = {k: np.zeros_like(val) for k, val in Pw.items()}
    ref, _, _ = pc.adam_step(Pw, G, zeros, dict(zeros), 1, lr=1e-2)
    got = P.gnn_unpack(w, 8)
    for k in pc.NAMES:
        assert np.allclose(got[k], ref[k], rtol=1e-6, atol=1e-7)


@gpu
@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_harvest_pairs_solve_correction_equation(rho):
    """k = 1, block 1: until the pair locks, Q = [x] exactly, so every pair
    must satisfy (I - x x^T)((C - rho theta) t - r) = 0 with t orthogonal
    to x (the target t = M r, minus the Jacobi-Davidson correction)."""
    need_gpu()
    import paper_1408_5535_amd as P
    A = wl.random_sparse(3000, 2000, 12, seed=1000)
    say("harvest 3000x2000 k=1 b=1 rho", rho)
    R, X, T, th, info = P.harvest(to_dev(A), 1, block=1, every=1, max_pairs=6, tol=1e-12,
                                  cg_tol=1e-10, shift_scale=rho)
    say("pairs", len(th), info["mv_prec"])
    assert len(th) >= 4
    R, X, T = as_np(R), as_np(X), as_np(T)
    for i in range(len(th)):
        r, x, t = R[i], X[i], T[i]
        assert abs(np.linalg.norm(x) - 1) < 1e-12
        v = A.T @ (A @ t) - rho * th[i] * t - r
        v -= x * (x @ v)
        assert abs(x @ t) < 1e-10 * np.linalg.norm(t)
        assert np.linalg.norm(v) < 1e-8 * np.linalg.norm(r)


@gpu
def test_svds_with_gnn_preconditioner_returns_definition():
    need_gpu()
    import paper_1408_5535_amd as P
    from oracle import dense
    A = wl.random_sparse(600, 400, 8, seed=2002)
    sig_ex, _, _ = dense.svd_extreme_dense(A, 4)
    an = float(np.linalg.norm(A.toarray(), 2))
    w = P.gnn_pack(wl.gnn_init_weights(32, seed=1))
    say("svds gnn 600x400 k=4")
    sig, U, V, info = P.svds_smallest(to_dev(A), 4, 1e-12, precond="gnn", gnn_weights=w,
                                      block=2, anorm=an)
    say(info)
    assert info["status"] == 0
    assert np.allclose(sig, sig_ex, rtol=1e-10)
    res = dense.triplet_residuals(A, sig, as_np(U), as_np(V))
    assert np.all(res <= 1e-12 * an)


@gpu
def test_learned_pipeline_training_gains():
    """The whole learned-preconditioner pipeline on a small member of the
    random family (6000 x 4000, 12 per row): harvest from stage-1 runs on
    four matrices, train with the library's forward/backward/Adam on the
    residual objective ||C t - r|| / ||r||, then solve two held-out matrices
    with no preconditioner, Jacobi and the networks.  Every arm must reach
    1e-12 ||A||.  Training must pay: from the Jacobi-equivalent start the
    trained network needs at most 0.8x the products of its start and of
    Jacobi on each held-out matrix; from the polynomial start (already far
    ahead of Jacobi) the trained network needs fewer products in total than
    its start.  Width 32, the network's size; times are printed."""
    need_gpu()
    from paper_1408_5535_amd import learned as L

    def make(seed):
        return wl.random_sparse(6000, 4000, 12, seed=seed)

    W = 32
    say("learned pipeline: starts")
    poly, hi, coeffs = L.poly_init(make(1000), width=W)
    jac = L.jacobi_init(W)
    say("bound", hi, "coefficients", coeffs)
    say("harvest")
    mats, graphs, pairs = L.harvest_family(range(1000, 1004), make, k=4, block=2, every=10,
                                           max_pairs=24, width=W)
    assert len(pairs) >= 40
    nets = {"poly": poly, "jac": jac}
    for name, ini, lr, ep in (("poly_trained", poly, 1e-4, 6), ("jac_trained", jac, 1e-3, 10)):
        say("train from", name, len(pairs), "pairs")
        w, hist, _ = L.train(graphs, pairs, width=W, epochs=ep, lr=lr, batch=8, init=ini,
                             loss_kind="residual")
        say("loss per epoch", hist)
        assert np.all(np.isfinite(hist)) and hist[-1] < hist[0]
        nets[name] = w
    del mats, graphs, pairs
    seeds = (2000, 2001)
    rows = L.evaluate(seeds, make, nets, width=W, k=4, block=2)
    for r in rows:
        say(r)
        assert r["status"] == 0 and r["max_res_over_norm"] <= 1e-12 * (1 + 1e-8)
    mv = {(r["seed"], r["method"]): r["mv"] for r in rows}
    say("products (none, jacobi, jacobi start, trained from it, polynomial, trained from it):",
        [(s, mv[(s, "none")], mv[(s, "jacobi")], mv[(s, "jac")], mv[(s, "jac_trained")],
          mv[(s, "poly")], mv[(s, "poly_trained")]) for s in seeds])
    say("seconds:", [(r["seed"], r["method"], round(r["seconds"], 3)) for r in rows])
    for s in seeds:
        assert mv[(s, "jac_trained")] <= 0.8 * mv[(s, "jacobi")]
        assert mv[(s, "jac_trained")] <= 0.8 * mv[(s, "jac")]
        assert mv[(s, "poly")] < mv[(s, "jacobi")]
    assert sum(mv[(s, "poly_trained")] for s in seeds) < sum(mv[(s, "poly")] for s in seeds)


@gpu
def test_gnn_forward_polynomial_weights_match_oracle():
    """The polynomial start (workloads.gnn_poly_weights) through the GPU
    forward equals the oracle's forward, i.e. the closed form
    D^-1/2 p(Ch) D^-1/2 r pinned in the oracle tests, in float32."""
    need_gpu()
    import paper_1408_5535_amd as P
    A, _, r, x, th, _ = _case(8)
    Pw = wl.gnn_poly_weights(wl.inverse_poly_coeffs(3.3, 3), 8)
    g = P.GnnGraph(to_dev(A), 8)
    t = as_np(g.forward(P.gnn_pack(Pw), _dev32(r), _dev32(x), th)).astype(np.float64)
    tref, _ = pc.forward(pc.Graph(A), Pw, r, x, th)
    err = np.max(np.abs(t - tref)) / np.max(np.abs(tref))
    say("poly weights max elementwise error / max |t|", err)
    assert err < 1e-5


@gpu
def test_jacobi_scaled_values_match_the_definition():
    """A D^-1/2 formed by the library: every value equals a_ij / ||A_:,j||."""
    need_gpu()
    import paper_1408_5535_amd as P
    A = wl.random_sparse(3000, 2000, 12, seed=1001)
    B = P.jacobi_scaled(to_dev(A))
    d = np.sqrt(np.asarray(A.multiply(A).sum(axis=0)).ravel())
    ref = A.data / d[A.indices]
    got = as_np(B.val)
    assert np.all(np.abs(got - ref) <= 4 * 2.0 ** -53 * np.abs(ref))
