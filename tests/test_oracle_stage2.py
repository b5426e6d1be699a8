"""Pins of the oracle's second stage (Section 3.2, Algorithm 2; Section 5.1,
Table 1) and of the JDQMR inner solver, against the paper's printed values,
closed forms, dense definitions and algebraic identities."""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import dense, jdqmr, phsvds as ph
from tests import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1_rows():
    rows = []
    with open(os.path.join(GOLDEN, "table1.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return np.array(rows)


# ------------------------------------------------------------- Table 1
def test_table1_end_to_end_with_jdqmr():
    """Section 5.1, Table 1: the ten clustered smallest singular values of
    diag([1e-14, 1e-12, 1e-8:1e-8:4e-8, 1e-3:1e-3:1]), block 2 in stage 1,
    no preconditioner, delta = 1e-15.  Every value is within 4x the error
    the paper prints, and every triplet meets the Section 5 test
    sqrt(||r_u||^2 + ||r_v||^2) <= delta ||A|| (the printed ||r_B|| are all
    below 1e-15 too)."""
    A = wl.table1_matrix()
    t = _table1_rows()
    exact, printed, rb = t[:, 0], t[:, 1], t[:, 2]
    out = ph.phsvds(A, 10, 1e-15, block=2, anorm=1.0, stage2_method="jdqmr")
    assert out["converged"]
    assert out["stats"].stage2_pairs == 10
    paper_err = np.abs(printed - exact)
    assert np.all(np.abs(out["sigma"] - exact) <= 4 * paper_err), (out["sigma"] - exact, paper_err)
    assert np.all(out["res"] <= 1e-15), out["res"]
    assert np.all(rb < 1e-15)
    # singular vectors: the coordinate vectors (A is diagonal), to the
    # Davis-Kahan bound sin(angle) <= ||r|| / gap
    d = A.diagonal()
    for i in range(10):
        gap = np.min(np.abs(np.delete(d, i) - d[i]))
        for W in (out["V"], out["U"]):
            sin = math.sqrt(max(0.0, 1.0 - W[i, i] ** 2))
            assert sin <= 2 * out["res"][i] / gap + 1e-14, (i, sin, out["res"][i] / gap)


def test_table1_gdk_budget_spent_reports_not_converged():
    """With GD+k in stage 2 the Table 1 run stalls (its refined vector cannot
    reach the 1e-14 eigenvector without inner solves); when the budget runs
    out, ``converged`` is False and some final residual exceeds tol ||A||."""
    A = wl.table1_matrix()
    out = ph.phsvds(A, 10, 1e-15, block=2, anorm=1.0, stage2_method="gdk", max_iters=6000)
    assert not out["converged"]
    assert np.any(out["res"] > 1e-15)


def test_converged_false_whenever_a_residual_exceeds_tol():
    """A stage-1-only solve cut short by the iteration budget is not
    converged, and its flag agrees with the final residuals."""
    A = wl.grid_gradient(12)
    an = cf.grid_norm(12)
    out = ph.phsvds(A, 6, 1e-12, block=2, anorm=an, max_iters=20)
    assert not out["converged"]
    assert np.any(out["res"] > 1e-12 * an)
    full = ph.phsvds(A, 6, 1e-12, block=2, anorm=an)
    assert full["converged"] == bool(np.all(full["res"] <= 1e-12 * an * (1 + 1e-8)))


# ------------------------------------------------------------- sQMR
def _sym_matrix(n, eigs, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * eigs) @ Q.T


@pytest.mark.parametrize("kind", ["spd", "indefinite"])
def test_sqmr_reaches_the_direct_solution(kind):
    n = 60
    eigs = np.linspace(0.5, 3.0, n) if kind == "spd" else np.concatenate(
        [-np.linspace(0.4, 2.0, n // 2), np.linspace(0.3, 2.5, n - n // 2)])
    M = _sym_matrix(n, eigs, 3)
    b = np.random.default_rng(4).standard_normal(n)
    t, s, steps, why = jdqmr.sqmr(lambda w: M @ w, b, maxit=400,
                                  stop=lambda k, t, s, tau: "done" if np.linalg.norm(s) < 1e-13 else None)
    assert why == "done"
    assert np.linalg.norm(t - np.linalg.solve(M, b)) < 1e-10 * np.linalg.norm(t)


def test_sqmr_residual_recurrence_and_quasi_residual_identity():
    """The recurrence residual s equals b - M t, and without a preconditioner
    its norm equals the quasi-residual tau (the CG residuals are mutually
    orthogonal, so the smoothing is exactly minimal), also when indefinite."""
    n = 50
    M = _sym_matrix(n, np.concatenate([-np.linspace(0.2, 1.5, 20), np.linspace(0.1, 2.0, 30)]), 5)
    b = np.random.default_rng(6).standard_normal(n)
    seen = []

    def stop(k, t, s, tau):
        seen.append((np.linalg.norm(s - (b - M @ t)), np.linalg.norm(s), tau))
        return None

    jdqmr.sqmr(lambda w: M @ w, b, maxit=12, stop=stop)
    for err, ns, tau in seen:
        assert err < 1e-12 * np.linalg.norm(b)
        assert abs(ns - tau) < 1e-10 * np.linalg.norm(b)


def test_sqmr_with_symmetric_preconditioner():
    n = 40
    M = _sym_matrix(n, np.concatenate([-np.linspace(1, 50, 15), np.linspace(2, 80, 25)]), 7)
    P = np.linalg.inv(M + 0.1 * _sym_matrix(n, np.linspace(-1, 1, n), 8))
    P = 0.5 * (P + P.T)
    b = np.random.default_rng(9).standard_normal(n)
    t, s, steps, why = jdqmr.sqmr(lambda w: M @ w, b, prec=lambda g: P @ g, maxit=200,
                                  stop=lambda k, t, s, tau: "ok" if np.linalg.norm(s) < 1e-12 * np.linalg.norm(b) else None)
    assert why == "ok" and steps < 40
    assert np.linalg.norm(b - M @ t) < 1e-11 * np.linalg.norm(b)


def test_eig_residual_estimate_is_the_explicit_residual():
    """The estimate of ||(B - mu) z|| / ||z|| for z = x + t at the best mu
    equals the explicit value (module notes of oracle.jdqmr)."""
    A = wl.random_sparse(40, 30, 5, seed=12).toarray()
    m, n = A.shape
    B = np.block([[np.zeros((n, n)), A.T], [A, np.zeros((m, m))]])
    rng = np.random.default_rng(13)
    x = rng.standard_normal(m + n)
    x /= np.linalg.norm(x)
    theta = float(x @ B @ x)
    r = B @ x - theta * x
    eta = theta * 0.9 + 0.01
    P = np.eye(m + n) - np.outer(x, x)
    t = P @ rng.standard_normal(m + n) * 0.3
    s = -r - P @ (B - eta * np.eye(m + n)) @ t
    est = jdqmr.eig_residual_estimate(r, theta, eta, t, s)
    z = x + t
    mus = np.linspace(-3, 3, 2001)
    mu_rq = float(z @ B @ z) / float(z @ z)
    explicit = np.linalg.norm(B @ z - mu_rq * z) / np.linalg.norm(z)
    assert abs(est - explicit) < 1e-12 * max(1.0, explicit)
    brute = min(np.linalg.norm(B @ z - mu * z) for mu in mus) / np.linalg.norm(z)
    assert est <= brute + 1e-12


def test_jd_correction_solves_the_projected_equation():
    A = wl.random_sparse(60, 40, 5, seed=14)
    Ad = A.toarray()
    m, n = Ad.shape
    B = np.block([[np.zeros((n, n)), Ad.T], [Ad, np.zeros((m, m))]])
    sig, U, V = dense.svd_extreme_dense(A, 2)
    rng = np.random.default_rng(15)
    x = np.concatenate([V[:, 0], U[:, 0]]) / math.sqrt(2) + 1e-3 * rng.standard_normal(m + n)
    x /= np.linalg.norm(x)
    theta = float(x @ B @ x)
    r = B @ x - theta * x
    Xl = np.concatenate([V[:, 1], U[:, 1]])[:, None] / math.sqrt(2)
    x = x - Xl[:, 0] * (Xl[:, 0] @ x)
    x /= np.linalg.norm(x)
    theta = float(x @ B @ x)
    r = B @ x - theta * x
    Q = np.column_stack([Xl, x])
    t, steps, why = jdqmr.jd_correction(lambda w: B @ w, x, r, theta, sig[0], Q, 0.0,
                                        max_inner=10 * (m + n))
    assert np.linalg.norm(Q.T @ t) < 1e-12
    P = np.eye(m + n) - Q @ Q.T
    lin = -r - P @ (B - sig[0] * np.eye(m + n)) @ P @ t
    # stopped by the shift-limited or stagnation rule, not by the cap
    assert why in ("linear", "stagnation", "converged")
    est = jdqmr.eig_residual_estimate(r, theta, sig[0], t, lin)
    assert est < 0.5 * np.linalg.norm(r)


# ------------------------------------------------------------- B-form Jacobi
def test_jacobi_precond_B_is_the_dense_block_operator():
    """P_B [f; g] = [M A^T g; A M f] with M = diag(C)^-1 (Section 4)."""
    A = wl.random_sparse(30, 20, 4, seed=16)
    Ad = A.toarray()
    d = ph.jacobi_diag(A)
    assert np.allclose(d, (Ad * Ad).sum(0), rtol=1e-14)
    M = np.diag(1.0 / d)
    PB = np.block([[np.zeros((20, 20)), M @ Ad.T], [Ad @ M, np.zeros((30, 30))]])
    st = ph.Stats()
    apply = ph.jacobi_precond_B(A, d, st)
    R = np.random.default_rng(17).standard_normal((50, 3))
    assert np.allclose(apply(R, None, None), PB @ R, rtol=1e-13, atol=1e-14)
    assert st.mv_prec == 3
    assert np.allclose(PB, PB.T)


@pytest.mark.parametrize("method", ["gdk", "jdqmr"])
def test_stage2_with_bform_jacobi_vs_closed_form(method):
    """A stage-2 solve that really applies the B-form Jacobi correction
    (mv_prec > 0): Givens-scrambled diagonal with sigma_1..3 = 1e-4..3e-4 at
    ||A|| = 1, so delta sigma / ||A|| < 10 eps and stage 1 stops at its floor.
    The result matches the closed form to 1e-10 relative."""
    n, m = 200, 240
    s = np.concatenate([[1e-4, 2e-4, 3e-4], np.linspace(0.05, 1.0, n - 3)])
    A, sig, U, V = wl.givens_scrambled(m, n, s, rot_left=int(0.7 * m), rot_right=int(0.7 * n),
                                       seed=2)
    out = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0, precond="jacobi", stage2_method=method)
    assert out["stats"].stage2_pairs == 3
    assert out["stats"].mv_prec > 0
    assert out["converged"]
    assert np.all(np.abs(out["sigma"] - sig[:3]) <= 1e-10 * sig[:3])
    assert np.all(out["res"] <= 1e-12)
    for i in range(3):
        assert abs(abs(out["V"][:, i] @ V[:, i]) - 1) < 1e-10


# ------------------------------------------------------------- random left vector
def test_random_left_vector_branch():
    """Section 3.3: a singular value so small that stage 1 gives no accuracy
    for u = A v / ||A v|| gets a random left vector, orthogonalised against
    the others; with it the JDQMR second stage still finds the triplet."""
    vals = np.concatenate([[1e-17, 1e-9], 1e-3 * np.arange(1, 301)])
    A = wl.diag_matrix(vals)
    an = float(vals.max())
    n = A.shape[1]
    Xl = np.zeros((n, 3))
    Xl[[0, 1, 2], [0, 1, 2]] = 1.0
    s, v, u = ph.transition_rr(A, Xl, np.zeros((n, 0)), 3, 3, an)
    assert s[0] <= 10 * ph.EPS64 * an < s[1]
    assert abs(np.linalg.norm(u[:, 0]) - 1) < 1e-14
    assert np.all(np.abs(u[:, 1:].T @ u[:, 0]) < 1e-14)
    # not A v / ||A v||: the e_1 component of a random unit vector is small
    assert abs(u[0, 0]) < 0.2
    Av = A @ v[:, 1]
    assert np.allclose(u[:, 1], Av / np.linalg.norm(Av), atol=1e-12)
    out = ph.phsvds(A, 3, 1e-12, block=2, anorm=an, stage2_method="jdqmr")
    assert out["converged"] and out["stats"].stage2_pairs >= 1
    assert np.all(np.abs(out["sigma"] - vals[:3]) <= out["res"] + 1e-30)
    assert np.all(out["res"] <= 1e-12 * an)


def test_triplet_residual_guard_rejects_unbalanced_vectors():
    """For sigma below the B threshold, [e_1; 0] passes ||B x - theta x|| <
    delta ||A|| / sqrt(2) but is no triplet; the lock test's triplet
    residual of the normalised halves rejects it, and equals sqrt(2) times
    the B residual for a balanced vector."""
    vals = np.array([1e-17, 0.5, 1.0])
    A = sp.diags(vals).tocsr()
    n = 3
    B = np.block([[np.zeros((n, n)), A.toarray()], [A.toarray(), np.zeros((n, n))]])
    x = np.zeros(6)
    x[0] = 1.0
    x[4] = 1e-12  # the bottom half is almost nothing but junk
    x /= np.linalg.norm(x)
    theta = float(x @ B @ x)
    assert np.linalg.norm(B @ x - theta * x) < 1e-12 / math.sqrt(2)
    assert ph._triplet_residual(x, B @ x, theta, n) > 0.1
    y = np.array([1.0, 0, 0.3, 1.0, 0, 0.3]) / math.sqrt(2.18)
    th = float(y @ B @ y)
    rb = np.linalg.norm(B @ y - th * y)
    assert abs(ph._triplet_residual(y, B @ y, th, n) - math.sqrt(2) * rb) < 1e-14


# ------------------------------------------------------------- refined projection
def test_refined_smallest_singular_value_nonincreasing_within_a_cycle():
    """Section 3.2: with a fixed shift, sigma_min(R) of W - s V can only fall
    as the search space grows (minimisation over nested spaces); it may
    rise only at restarts and locks."""
    A = wl.random_sparse(200, 120, 6, seed=20)
    sig, U, V = dense.svd_extreme_dense(A, 2)
    rng = np.random.default_rng(21)
    v0 = V + 1e-4 * rng.standard_normal(V.shape)
    u0 = A @ v0
    u0 /= np.linalg.norm(u0, axis=0)
    an = np.linalg.norm(A.toarray(), 2)
    tr = []
    st = ph.Stats()
    ph.stage2_refined(A, sig * (1 + 1e-6), v0, u0, 1e-12, an, 1, 20, 12, stats=st, trace=tr)
    grew = 0
    for a, b in zip(tr, tr[1:]):
        if b[1] == a[1] + 1 and b[5] == a[5]:
            grew += 1
            assert b[4] <= a[4] * (1 + 1e-10) + 1e-15 * an
    assert grew >= 5


# ------------------------------------------------------------- boundary forms
def test_resume_from_saved_stage1_output_vs_closed_form():
    """Algorithm 2 step 1 inputs given directly (saved first-stage vectors
    and shifts): the second stage alone reaches the closed form."""
    n, m = 200, 240
    s = np.concatenate([[1e-4, 2e-4, 3e-4], np.linspace(0.05, 1.0, n - 3)])
    A, sig, U, V = wl.givens_scrambled(m, n, s, rot_left=int(0.7 * m), rot_right=int(0.7 * n),
                                       seed=2)
    rng = np.random.default_rng(22)
    V0 = V[:, :3] + 1e-7 * rng.standard_normal((n, 3))
    shifts = sig[:3] * (1 + 1e-9)
    out = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0, init_V=V0, shifts=shifts)
    assert out["converged"] and out["stats"].stage2_pairs == 3
    assert out["stats"].mv_stage1 == 0
    assert np.all(np.abs(out["sigma"] - sig[:3]) <= 1e-10 * sig[:3])
    # left vectors of the seeds: A v / ||A v|| (no tiny shifts here)
    v0, u0 = ph.resume_seeds(A, V0, shifts, 1.0)
    Av = A @ (V0 / np.linalg.norm(V0, axis=0))
    assert np.allclose(u0, Av / np.linalg.norm(Av, axis=0), atol=1e-14)


def test_callable_preconditioner_and_its_bform():
    """A caller's C-preconditioner (here diag(C)^-1 as a callable): stage 1
    uses it directly, stage 2 its B-form [M A^T g; A M f]; the result is the
    dense SVD, and the B-form equals the dense block operator."""
    A = wl.random_sparse(240, 160, 6, seed=23)
    d = ph.jacobi_diag(A)
    calls = []

    def M(R, theta):
        calls.append(np.asarray(theta).copy())
        return R / d[:, None]

    sig, U, V = dense.svd_extreme_dense(A, 3)
    an = np.linalg.norm(A.toarray(), 2)
    out = ph.phsvds(A, 3, 1e-12, block=1, anorm=an, precond=M, stage2="force",
                    stage2_method="gdk")
    assert out["converged"] and calls
    assert np.all(np.abs(out["sigma"] - sig) <= 1e-10 * sig)
    n, m = 160, 240
    Ad = A.toarray()
    PB = np.block([[np.zeros((n, n)), np.diag(1 / d) @ Ad.T], [Ad @ np.diag(1 / d), np.zeros((m, m))]])
    st = ph.Stats()
    # the B-form the oracle builds from M, applied to random blocks
    R = np.random.default_rng(24).standard_normal((n + m, 2))
    f, g = R[:n], R[n:]
    got = np.vstack([M(A.T @ g, [0, 0]), A @ M(f, [0, 0])])
    assert np.allclose(got, PB @ R, rtol=1e-13, atol=1e-14)
