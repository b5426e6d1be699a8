"""Edge cases of the solver through the C ABI, against a dense SVD of the
same matrix (LAPACK through NumPy) and the CPU oracle: all n triplets of a
small matrix, a block wider than the remaining targets, square and very
tall matrices, zero rows, a singular value of multiplicity three, and a
space too small for the block.  Bars as for the other solver tests: sigma
within 1e-10 relative, residuals within tol ||A||, orthonormal V."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import dense, phsvds as ph
from tests.gpu_util import as_np, gpu, need_gpu, say, to_dev


def _check(A, k, b, tol=1e-12):
    import paper_1408_5535_amd as P
    Ad = A.toarray()
    s_all = np.linalg.svd(Ad, compute_uv=False)
    an = float(s_all[0])
    ex = np.sort(s_all)[:k]
    say(f"{A.shape[0]} x {A.shape[1]}, nnz {A.nnz}, k={k}, b={b}")
    sig, U, V, info = P.svds_smallest(to_dev(A), k, tol, block=b, anorm=an)
    say({q: info[q] for q in ("status", "mv_total", "stage2_pairs")})
    assert info["status"] == 0
    assert np.all(np.abs(sig - ex) <= 1e-10 * ex), (sig, ex)
    res = dense.triplet_residuals(A, sig, as_np(U), as_np(V))
    assert np.all(res <= tol * an), res
    Vn = as_np(V)
    assert np.linalg.norm(Vn.T @ Vn - np.eye(k)) < 1e-10
    out = ph.phsvds(A, k, tol, block=b, anorm=an)
    assert out["converged"] and np.all(np.abs(out["sigma"] - ex) <= 1e-10 * ex)
    return sig, as_np(U), Vn


@gpu
@pytest.mark.parametrize("m,n,k,b", [(12, 6, 6, 1), (12, 6, 3, 2), (30, 30, 5, 2),
                                     (5000, 10, 4, 2)])
def test_small_square_and_very_tall(m, n, k, b):
    """k = n (every triplet; the basis is capped at n), a block wider than
    the targets left, a square matrix, and m = 500 n."""
    need_gpu()
    _check(wl.random_sparse(m, n, min(4, n), seed=3), k, b)


@gpu
def test_zero_rows():
    """Rows with no entries (empty CSR rows, also in the device transpose)
    leave the singular values unchanged."""
    need_gpu()
    A0 = wl.random_sparse(200, 60, 5, seed=4).tocsr()
    A = sp.vstack([A0[:100], sp.csr_matrix((50, 60)), A0[100:], sp.csr_matrix((7, 60))]).tocsr()
    assert np.sum(np.diff(A.indptr) == 0) >= 57
    _check(A, 4, 2)


@gpu
def test_singular_value_of_multiplicity_three():
    """sigma = 0.5 three times (then 1, 1.01, ...), Givens-scrambled: the
    three values to 1e-10 and the computed right vectors span the exact
    three-dimensional singular subspace (largest principal angle < 1e-8)."""
    need_gpu()
    n, m = 120, 150
    s = np.concatenate([[0.5, 0.5, 0.5], np.linspace(1.0, 2.0, n - 3)])
    A, sx, Ux, Vx = wl.givens_scrambled(m, n, s, rot_left=int(0.7 * m), rot_right=int(0.7 * n),
                                        seed=6)
    sig, U, V = _check(A, 4, 2)
    Q = np.linalg.qr(V[:, :3])[0]
    # sine of the largest principal angle: ||(I - Q Q^T) V_exact||_2 (the
    # cosine route loses half the digits near 1)
    E = Vx[:, :3] - Q @ (Q.T @ Vx[:, :3])
    sine = float(np.linalg.norm(E, 2))
    say("largest principal angle, sine", sine)
    assert sine < 1e-8


@gpu
def test_space_too_small_for_the_block_is_einval():
    """n = 10 with block 4: a basis capped at n cannot hold a restart plus a
    block (n < 3b); both sides refuse it."""
    need_gpu()
    import paper_1408_5535_amd as P
    A = wl.random_sparse(40, 10, 4, seed=3)
    with pytest.raises(RuntimeError, match=r"\(-1\)"):
        P.svds_smallest(to_dev(A), 4, 1e-12, block=4)
    with pytest.raises(ValueError):
        ph.phsvds(A, 4, 1e-12, block=4)


@gpu
def test_initial_columns_dependent_on_the_basis_are_replaced():
    """A caller's start block [x, y, x, z] at block 2: after the first chunk
    [x, y] the repeated x of the second chunk has no component left outside
    the basis, so Gram-Schmidt replaces it by a seeded random vector
    (stats dep_cols) and the solve still finds the closed-form values."""
    need_gpu()
    import torch

    import paper_1408_5535_amd as P
    A = wl.grid_gradient(16)
    N = 16
    i = np.arange(1, N + 1)
    s2 = 4 * np.sin(i * np.pi / (2 * (N + 1))) ** 2
    ex = np.sort(np.sqrt((s2[:, None] + s2[None, :]).ravel()))[:4]
    r = np.random.default_rng(5)
    x, y, z = (r.standard_normal(A.shape[1]) for _ in range(3))
    X0 = np.column_stack([x, y, x, z])
    say("dependent start columns", A.shape, "k0", X0.shape[1])
    sig, U, V, info = P.svds_smallest(to_dev(A), 4, 1e-12, block=2, anorm=float(np.sqrt(8.0)),
                                      init_V=torch.tensor(X0))
    say({q: info[q] for q in ("status", "mv_total", "dep_cols")})
    assert info["dep_cols"] >= 1
    assert info["status"] == 0
    assert np.all(np.abs(sig - ex) <= 1e-10 * ex), (sig, ex)
    res = dense.triplet_residuals(A, sig, as_np(U), as_np(V))
    assert np.all(res <= 1e-12 * np.sqrt(8.0)), res


@gpu
@pytest.mark.parametrize("fp32", [False, True])
def test_power_law_rows_left_vectors_in_the_callers_order(fp32):
    """Rows of seven length classes (power law, 2000 x 1000): the solver
    keeps the row space in bin order internally; sigma against LAPACK and
    the oracle, residuals within tol ||A||, and U against LAPACK's left
    vectors up to sign, in the caller's row order."""
    need_gpu()
    import paper_1408_5535_amd as P
    A = wl.powerlaw_sparse(2000, 1000, mean=10, kmax=200, seed=41)
    assert len(np.unique(np.minimum(np.ceil(np.log2(np.maximum(np.diff(A.indptr), 4) / 4)),
                                     6))) >= 5
    Ud, s_all, Vdt = np.linalg.svd(A.toarray(), full_matrices=False)
    an = float(s_all[0])
    k = 4
    ex, Uex = s_all[::-1][:k], Ud[:, ::-1][:, :k]
    say("power-law rows", A.shape, "fp32", fp32)
    sig, U, V, info = P.svds_smallest(to_dev(A), k, 1e-12, block=2, anorm=an,
                                      stage1_fp32=fp32)
    say({q: info[q] for q in ("status", "mv_total", "stage2_pairs")})
    assert info["status"] == 0
    assert np.all(np.abs(sig - ex) <= 1e-10 * ex), (sig, ex)
    Un = as_np(U)
    res = dense.triplet_residuals(A, sig, Un, as_np(V))
    assert np.all(res <= 1e-12 * an), res
    assert np.all(np.abs(np.abs(np.sum(Un * Uex, axis=0)) - 1.0) <= 1e-9), Un.T @ Uex
    out = ph.phsvds(A, k, 1e-12, block=2, anorm=an)
    assert out["converged"] and np.all(np.abs(out["sigma"] - sig) <= 1e-10 * ex)


@gpu
def test_power_law_rows_solve_is_deterministic():
    """Two solves of the same power-law matrix (rows of seven length
    classes, so the row space is in bin order) give bit-identical sigma,
    U, V and product counts: the bin order depends only on the row lengths
    and every sum has a fixed order."""
    need_gpu()
    import paper_1408_5535_amd as P
    A = wl.powerlaw_sparse(2000, 1000, mean=10, kmax=200, seed=41)
    an = float(np.linalg.norm(A.toarray(), 2))
    Ad = to_dev(A)
    say("deterministic power-law solve", A.shape)
    out = [P.svds_smallest(Ad, 4, 1e-12, block=2, anorm=an) for _ in range(2)]
    (s1, U1, V1, i1), (s2, U2, V2, i2) = out
    assert i1["mv_total"] == i2["mv_total"] and i1["status"] == i2["status"] == 0
    assert np.array_equal(s1, s2)
    assert np.array_equal(as_np(U1), as_np(U2)) and np.array_equal(as_np(V1), as_np(V2))
