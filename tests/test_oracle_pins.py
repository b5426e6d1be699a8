"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: LAPACK,
closed-form spectra, the paper's printed values, algebraic identities of
Section 3.1, or published generator outputs.
"""
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import dense, phsvds as ph, rng
from tests import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ----------------------------------------------------------------- dense SVD
@pytest.mark.parametrize("shape", [(5, 3), (40, 25), (60, 60), (90, 12)])
def test_jacobi_svd_matches_lapack(shape):
    r = np.random.default_rng(sum(shape))
    A = r.standard_normal(shape) * np.logspace(0, -6, shape[1])[None, :]
    U, s, V = dense.jacobi_svd(A)
    s_ref = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s, s_ref, rtol=1e-12, atol=0)
    assert np.linalg.norm(U.T @ U - np.eye(shape[1])) < 1e-13
    assert np.linalg.norm(V.T @ V - np.eye(shape[1])) < 1e-13
    assert np.linalg.norm(A @ V - U * s) < 1e-13 * s[0]


def test_jacobi_svd_grid_closed_form():
    N = 6
    A = wl.grid_gradient(N).toarray()
    assert A.shape == (2 * N * (N + 1), N * N)
    _, s, _ = dense.jacobi_svd(A)
    assert np.allclose(np.sort(s), cf.grid_sigmas(N), rtol=1e-13)


def test_givens_generator_closed_form():
    A, sig, U, V = wl.givens_scrambled(60, 50, np.logspace(-3, 0, 50), rot_left=200, rot_right=150, seed=4)
    Ad = A.toarray()
    # A v_i = sigma_i u_i and A^T u_i = sigma_i v_i with orthonormal U, V
    assert np.linalg.norm(Ad @ V - U * sig) < 1e-13
    assert np.linalg.norm(Ad.T @ U - V * sig) < 1e-13
    assert np.linalg.norm(U.T @ U - np.eye(50)) < 1e-13
    s = np.linalg.svd(Ad, compute_uv=False)
    assert np.allclose(np.sort(s), sig, rtol=1e-11)


def test_svd_extreme_dense_definition():
    A = wl.random_sparse(120, 80, 6, seed=5)
    sig, U, V = dense.svd_extreme_dense(A, 4)
    s_ref = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:4]
    assert np.allclose(sig, s_ref, rtol=1e-12)
    assert np.all(dense.triplet_residuals(A, sig, U, V) < 1e-13)


# ------------------------------------------------------------- generators
def test_splitmix64_published_first_output():
    (row,) = _load_table("splitmix64.txt")
    z = rng.splitmix64(np.array([int(row[0])], dtype=np.uint64))
    assert int(z[0]) == int(row[1], 16)


def test_table1_matrix_matches_paper_definition():
    A = wl.table1_matrix()
    assert A.shape == (1006, 1006)
    rows = _load_table("table1.txt")
    exact = np.array([float(r[0]) for r in rows])
    assert np.allclose(np.sort(A.diagonal())[:10], exact, rtol=4e-16, atol=0)


def test_zipf_shift_gives_mean():
    q = wl.zipf_shift_for_mean(10.0, 2000, 2.0)
    p = wl._zipf_pmf(2000, 2.0, q)
    assert abs((np.arange(1, 2001) * p).sum() - 10.0) < 1e-9
    assert 0.9 < q < 1.05


def test_jacobi_diag_is_column_norms():
    A = wl.random_sparse(50, 30, 5, seed=2)
    assert np.allclose(ph.jacobi_diag(A), (A.toarray() ** 2).sum(0), rtol=1e-14)


# ---------------------------------------------------------- Section 3.1
def test_residual_identities_section31():
    """With u = A v / s: r_v = 0, r_C = s r_u and ||r_u|| = ||r_C||/s = sqrt(2)||r_B||."""
    A = wl.random_sparse(150, 100, 8, seed=9)
    X0 = wl.initial_block(100, 2, 3)
    pmax, pmin = ph.basis_sizes(3, 2)
    Xl, th, _, _, _ = ph.stage1_gdk(A, 3, 1e-6, 2, pmax, pmin, X0)
    for i in range(3):
        v = Xl[:, i]
        v = v / np.linalg.norm(v)
        s = math.sqrt(th[i])
        u = A @ v / s
        rv = A @ v - s * u
        ru = A.T @ u - s * v
        rC = A.T @ (A @ v) - s * s * v
        x = np.concatenate([v, u])
        rB = np.concatenate([A.T @ u, A @ v]) - s * x
        rB = rB / np.linalg.norm(x)
        assert np.linalg.norm(rv) < 1e-14
        assert np.allclose(rC, s * ru, atol=1e-13 * s)
        assert math.isclose(np.linalg.norm(ru), np.linalg.norm(rC) / s, rel_tol=1e-8)
        assert math.isclose(np.linalg.norm(ru), math.sqrt(2) * np.linalg.norm(rB), rel_tol=1e-8)


def test_dynamic_tolerance_and_stage2_entry():
    """delta_C = max(delta s_i / s_n, eps) (Section 3.1): the largest pairs
    never need stage 2; pairs with delta s_i/s_n < eps do."""
    N = 8
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    out = ph.phsvds(A, 4, 1e-12, which="largest", block=2, anorm=an)
    assert out["stats"].stage2_pairs == 0 and out["stats"].mv_stage2 == 0
    s = cf.grid_sigmas(N)
    # delta s_1/||A|| = 1e-12 * 0.3 / 2.8 ~ 1e-13 >> 10 eps: stage 1 suffices
    out = ph.phsvds(A, 4, 1e-12, block=2, anorm=an)
    assert out["stats"].stage2_pairs == 0
    # delta = 1e-16: every smallest pair needs stage 2
    out = ph.phsvds(A, 2, 1e-15, block=2, anorm=an, stage2="auto")
    assert out["stats"].stage2_pairs == 2
    assert np.allclose(out["sigma"], s[:2], rtol=1e-13)


# --------------------------------------------------------- full method
def _check_against_closed_form(out, exact, anorm, tol=1e-12, rel=1e-10):
    sig = out["sigma"]
    assert out["converged"]
    assert np.all(np.abs(sig - exact) <= rel * exact), (sig, exact)
    assert np.all(out["res"] <= tol * anorm), out["res"]
    # Bauer-Fike (Section 3.1): |sigma - sigma_exact| <= residual
    assert np.all(np.abs(sig - exact) <= out["res"] + 4 * ph.EPS64 * anorm)


def test_oracle_grid_smallest_closed_form():
    N = 16
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    out = ph.phsvds(A, 10, 1e-12, block=4, anorm=an)
    ex = cf.grid_sigmas(N)[:10]
    _check_against_closed_form(out, ex, an)
    # right singular subspace of each complete cluster (closed-form sine vectors)
    lam = cf.grid_lambdas(N)
    pairs = sorted(((lam[i] + lam[j], i + 1, j + 1) for i in range(N) for j in range(N)))[:10]
    for g in cf.clusters(ex):
        if g[-1] == 9 and abs(ex[9] - cf.grid_sigmas(N)[10]) < 1e-8 * ex[9]:
            continue
        Vex = np.column_stack([np.kron(cf.grid_sine(N, pairs[t][2]), cf.grid_sine(N, pairs[t][1])) for t in g])
        assert cf.principal_angles(out["V"][:, g], Vex) < 1e-8


def test_oracle_grid_largest_closed_form():
    N = 16
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    out = ph.phsvds(A, 10, 1e-12, which="largest", block=4, anorm=an)
    ex = cf.grid_sigmas(N)[::-1][:10]
    _check_against_closed_form(out, ex, an)


def test_oracle_forced_stage2_matches():
    N = 16
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    out = ph.phsvds(A, 6, 1e-12, block=2, anorm=an, stage2="force")
    assert out["stats"].stage2_pairs == 6
    _check_against_closed_form(out, cf.grid_sigmas(N)[:6], an)


def test_oracle_givens_two_stage_closed_form():
    n, m = 200, 240
    s = np.concatenate([[1e-3, 2e-3, 3e-3, 4e-3, 5e-3], np.linspace(0.05, 1.0, n - 5)])
    A, sig, U, V = wl.givens_scrambled(m, n, s, rot_left=int(0.7 * m), rot_right=int(0.7 * n), seed=1)
    out = ph.phsvds(A, 5, 1e-12, block=1, anorm=1.0)
    assert out["stats"].stage2_pairs >= 1
    _check_against_closed_form(out, sig[:5], 1.0)
    for i in range(5):
        assert abs(abs(out["V"][:, i] @ V[:, i]) - 1) < 1e-12
        assert abs(abs(out["U"][:, i] @ U[:, i]) - 1) < 1e-12


def test_oracle_random_sparse_vs_dense_definition():
    A = wl.random_sparse(300, 200, 8, seed=21)
    sig, U, V = dense.svd_extreme_dense(A, 4)
    an = np.linalg.norm(A.toarray(), 2)
    out = ph.phsvds(A, 4, 1e-12, block=2, anorm=an, precond="jacobi")
    _check_against_closed_form(out, sig, an)
    for i in range(4):
        assert abs(abs(out["V"][:, i] @ V[:, i]) - 1) < 1e-10


def test_stage2_exact_seeds_lock_immediately():
    """With exact shifts and vectors the refined vector is the eigenvector
    (sigma_min(R) = 0) and each target locks in one iteration."""
    A = wl.table1_matrix()
    d = A.diagonal()
    idx = np.argsort(d)[:4]
    n = A.shape[0]
    V = np.zeros((n, 4))
    V[idx, np.arange(4)] = 1.0
    st = ph.Stats()
    th, X = ph.stage2_refined(A, d[idx], V, V.copy(), 1e-15, 1.0, 1, 35, 21, stats=st)
    assert np.allclose(th, d[idx], rtol=1e-13)
    assert st.iters2 == 4


def test_transition_rr_improves_ritz_values():
    """Post-processing RR (Section 3.1): the Ritz values over span(Z) are
    at least as small as the Rayleigh quotients of the input vectors."""
    A = wl.random_sparse(200, 120, 6, seed=33)
    sig, U, V = dense.svd_extreme_dense(A, 3)
    r = np.random.default_rng(0)
    Xl = V + 1e-4 * r.standard_normal(V.shape)
    Xl /= np.linalg.norm(Xl, axis=0)
    rq = np.sort(np.sqrt(np.einsum("ij,ij->j", A @ Xl, A @ Xl)))
    s_rr, v_rr, u_rr = ph.transition_rr(A, Xl, np.zeros((120, 0)), 3, 3, 1.0)
    assert s_rr[0] <= rq[0] * (1 + 1e-14)
    # RR preserves the trace of the projection: sum theta_i = trace(Z^T C Z)
    Z, _ = np.linalg.qr(Xl)
    AZ = A @ Z
    assert math.isclose(np.sum(s_rr ** 2), float(np.einsum("ij,ij->", AZ, AZ)), rel_tol=1e-13)
    # Courant-Fischer: each Ritz value bounds the exact one from above
    assert np.all(s_rr >= sig * (1 - 1e-13))


def test_table1_stage1_and_rr_accuracy():
    """Table 1 matrix: stage 1 (block 2) plus the transition RR already give
    the well-separated values to the accuracy the paper prints."""
    A = wl.table1_matrix()
    rows = _load_table("table1.txt")
    exact = np.array([float(r[0]) for r in rows])
    printed = np.array([float(r[1]) for r in rows])
    X0 = wl.initial_block(A.shape[1], 2, 2)
    Xl, th, Vr, sn2, info = ph.stage1_gdk(A, 10, 1e-15, 2, 35, 21, X0, anorm=1.0)
    assert info["converged"]
    s_rr, _, _ = ph.transition_rr(A, Xl, Vr, 10, 21, 1.0)
    paper_err = np.abs(printed - exact)
    # sigma >= 1e-8: at least as accurate as the paper's final values
    assert np.all(np.abs(s_rr[2:] - exact[2:]) <= np.maximum(paper_err[2:], 1e-18) * 4)


def test_basis_capped_at_n_and_every_triplet():
    """p_max is capped at n; with k = n the oracle returns every singular
    value (dense SVD); n < 3b is refused."""
    assert ph.basis_sizes(6, 1, n=6) == (6, 4)
    A = wl.random_sparse(12, 6, 4, seed=3)
    out = ph.phsvds(A, 6, 1e-12, block=1)
    s = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))
    assert out["converged"] and np.allclose(out["sigma"], s, rtol=1e-12, atol=0)
    with pytest.raises(ValueError):
        ph.basis_sizes(4, 4, n=10)


def test_triplet_residual_checker_closed_forms():
    """The residual every solver test applies, pinned by hand-made triplets
    of A = [diag(s); 0] (m > n): exact triplets give 0; moving u by delta
    along another coordinate j gives delta sqrt(s_i^2 + s_j^2) for j < n
    and delta s_i for a zero row j >= n (where A^T e_j = 0, which a
    transposition mistake would miss); flipping the sign of u gives
    2 sqrt(2) s_i (which a sign mistake would not)."""
    import scipy.sparse as sp
    m, n = 9, 5
    s = np.array([0.3, 1.0, 2.0, 2.5, 4.0])
    A = sp.csr_matrix(np.vstack([np.diag(s), np.zeros((m - n, n))]))
    U, V = np.eye(m)[:, :n], np.eye(n)
    assert np.all(dense.triplet_residuals(A, s, U, V) == 0.0)
    delta, i = 1e-3, 1
    for j, want in ((3, delta * np.hypot(s[i], s[3])), (7, delta * s[i])):
        u = np.eye(m)[:, i] + delta * np.eye(m)[:, j]
        got = dense.triplet_residuals(A, [s[i]], u[:, None], V[:, i:i + 1])[0]
        assert abs(got - want) <= 1e-15, (j, got, want)
    got = dense.triplet_residuals(A, s, -U, V)
    assert np.allclose(got, 2 * np.sqrt(2) * s, rtol=1e-15)
