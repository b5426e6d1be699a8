"""The C-ABI boundary on the GPU: the transposed product, CSR validation,
k up to 64, the caller's preconditioner (USER) and resuming the second stage
from saved first-stage output.  Each is checked against SciPy, closed forms
or the CPU oracle."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as wl
from oracle import dense, phsvds as ph
from tests import closed_forms as cf
from tests.gpu_util import as_np, gpu, need_gpu, say, to_dev


def _err_bound(A, X, trans, eps):
    """|op(A)| |X| * n_row * eps: the forward-error bound of a dot product."""
    Aa = abs(A.T if trans else A).tocsr()
    rowlen = np.diff(Aa.indptr).max()
    return (Aa @ np.abs(X)) * (rowlen + 2) * eps


@gpu
@pytest.mark.parametrize("family", ["random", "powerlaw"])
@pytest.mark.parametrize("b", [1, 4, 8])
@pytest.mark.parametrize("trans", [False, True])
def test_spmm_op_both_directions_vs_scipy(family, b, trans):
    need_gpu()
    import paper_1408_5535_amd as P
    A = wl.random_sparse(3000, 2000, 9, seed=31) if family == "random" else \
        wl.powerlaw_sparse(3000, 2000, kmax=300, seed=32)
    rows_in = A.shape[0] if trans else A.shape[1]
    X = np.random.default_rng(33).standard_normal((rows_in, b))
    ref = (A.T if trans else A) @ X
    say("spmm_op", family, "b", b, "trans", trans)
    Y = as_np(P.spmm_op(to_dev(A), torch.tensor(X, device="cuda").contiguous(), trans=trans))
    assert np.all(np.abs(Y - ref) <= _err_bound(A, X, trans, 2.0 ** -53) + 1e-300)
    X32 = X.astype(np.float32)
    Y32 = as_np(P.spmm_op(to_dev(A), torch.tensor(X32, device="cuda").contiguous(), trans=trans))
    ref32 = (A.T if trans else A) @ X32.astype(np.float64)
    assert np.all(np.abs(Y32 - ref32) <= _err_bound(A, X32.astype(np.float64), trans, 2.0 ** -23)
                  * 2 + 1e-30)


def _bad_csr(kind):
    A = wl.random_sparse(60, 40, 5, seed=34).tocsr()
    A.sort_indices()
    rp, ci, va = A.indptr.astype(np.int64).copy(), A.indices.astype(np.int32).copy(), A.data.copy()
    if kind == "unsorted":
        ci[rp[3]], ci[rp[3] + 1] = ci[rp[3] + 1], ci[rp[3]]
    elif kind == "duplicate":
        ci[rp[5] + 1] = ci[rp[5]]
    elif kind == "rowptr":
        rp[-1] -= 1
    elif kind == "range":
        ci[rp[7]] = 40
    import paper_1408_5535_amd as P
    return P.DeviceCSR(60, 40, torch.tensor(rp, device="cuda"), torch.tensor(ci, device="cuda"),
                       torch.tensor(va, device="cuda"))


@gpu
@pytest.mark.parametrize("kind", ["unsorted", "duplicate", "rowptr", "range"])
def test_malformed_csr_is_einval(kind):
    need_gpu()
    import paper_1408_5535_amd as P
    D = _bad_csr(kind)
    say("malformed CSR", kind)
    with pytest.raises(RuntimeError, match=r"\(-1\)"):
        P.spmm_op(D, torch.ones((60, 2), dtype=torch.float64, device="cuda"), trans=True)
    with pytest.raises(RuntimeError, match=r"\(-1\)"):
        P.svds_smallest(D, 2, 1e-10)


@gpu
@pytest.mark.parametrize("k", [40, 64])
def test_many_triplets_closed_form(k):
    """k beyond the old 24 up to 64 (grid N = 24, n = 576): sigma against
    the closed form, float64 residuals recomputed on the host."""
    need_gpu()
    import paper_1408_5535_amd as P
    N = 24
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    say("grid N=24 k", k)
    sig, U, V, info = P.svds_smallest(to_dev(A), k, 1e-12, block=4, anorm=an)
    say({q: info[q] for q in ("status", "mv_total", "iters1", "stage2_pairs")})
    assert info["status"] == 0
    ex = cf.grid_sigmas(N)[:k]
    assert np.all(np.abs(sig - ex) <= 1e-10 * ex)
    res = dense.triplet_residuals(A, sig, as_np(U), as_np(V))
    assert np.all(res <= 1e-12 * an)
    Vn = as_np(V)
    assert np.linalg.norm(Vn.T @ Vn - np.eye(k)) < 1e-9


def _givens_small():
    n, m = 200, 240
    s = np.concatenate([[1e-4, 2e-4, 3e-4], np.linspace(0.05, 1.0, n - 3)])
    return wl.givens_scrambled(m, n, s, rot_left=int(0.7 * m), rot_right=int(0.7 * n), seed=2)


@gpu
@pytest.mark.parametrize("method", ["gdk", "jdqmr"])
def test_user_preconditioner_vs_oracle(method):
    """USER: the caller's M = diag(C)^-1, written with torch on the pointers
    the library hands over, in both stages (stage 2: its B-form)."""
    need_gpu()
    import paper_1408_5535_amd as P
    A, sigx, Ux, Vx = _givens_small()
    D = to_dev(A)
    d64 = torch.zeros(A.shape[1], dtype=torch.float64, device="cuda").index_add_(
        0, D.colind.long(), D.val * D.val)
    seen = {"calls": 0, "fp64": set()}

    def apply(R, T, theta, fp64):
        seen["calls"] += 1
        seen["fp64"].add(fp64)
        T.copy_(R / (d64 if fp64 else d64.float())[None, :])

    say("USER preconditioner, givens 1e-4, stage 2", method)
    X0 = torch.tensor(wl.initial_block(A.shape[1], 1, 2))
    sig, U, V, info = P.svds_smallest(D, 3, 1e-12, block=1, anorm=1.0, precond="user",
                                      user_apply=apply, init_block=X0, stage2_method=method)
    say({q: info[q] for q in ("status", "mv_total", "mv_prec", "stage2_pairs")}, seen["calls"])
    assert info["status"] == 0 and seen["calls"] > 0 and seen["fp64"] == {True}
    assert info["stage2_pairs"] == 3 and info["mv_prec"] > 0
    assert np.all(np.abs(sig - sigx[:3]) <= 1e-10 * sigx[:3])
    assert np.all(dense.triplet_residuals(A, sig, as_np(U), as_np(V)) <= 1e-12)
    d = ph.jacobi_diag(A)
    out = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0, precond=lambda R, th: R / d[:, None],
                    stage2_method=method)
    assert out["converged"]
    ratio = info["mv_total"] / out["stats"].mv_total
    say("MV gpu/oracle", ratio)
    assert 0.5 <= ratio <= 2.0


@gpu
def test_user_preconditioner_float32_stage1_and_error_return():
    need_gpu()
    import paper_1408_5535_amd as P
    A, sigx, Ux, Vx = _givens_small()
    D = to_dev(A)
    d64 = torch.zeros(A.shape[1], dtype=torch.float64, device="cuda").index_add_(
        0, D.colind.long(), D.val * D.val)
    kinds = set()

    def apply(R, T, theta, fp64):
        kinds.add(fp64)
        T.copy_(R / (d64 if fp64 else d64.float())[None, :])

    say("USER preconditioner with a float32 first stage")
    sig, U, V, info = P.svds_smallest(D, 3, 1e-12, block=1, anorm=1.0, precond="user",
                                      user_apply=apply, stage1_fp32=True, fp64_continue=False)
    assert info["status"] == 0 and kinds == {False, True}
    assert np.all(np.abs(sig - sigx[:3]) <= 1e-10 * sigx[:3])

    def failing(R, T, theta, fp64):
        raise ValueError("no preconditioner today")

    with pytest.raises(RuntimeError, match=r"\(-5\)"):
        P.svds_smallest(D, 3, 1e-12, block=1, anorm=1.0, precond="user", user_apply=failing)


@gpu
@pytest.mark.parametrize("method", ["gdk", "jdqmr"])
def test_resume_second_stage_from_saved_output(method):
    """init_V + shifts: the first stage is skipped and the saved vectors and
    shifts seed Algorithm 2 directly; against the closed form and the
    oracle's resume."""
    need_gpu()
    import paper_1408_5535_amd as P
    A, sigx, Ux, Vx = _givens_small()
    V0 = Vx[:, :3] + 1e-7 * np.random.default_rng(35).standard_normal((A.shape[1], 3))
    shifts = sigx[:3] * (1 + 1e-9)
    say("resume stage 2", method)
    sig, U, V, info = P.svds_smallest(to_dev(A), 3, 1e-12, block=1, anorm=1.0,
                                      init_V=torch.tensor(V0), shifts=list(shifts),
                                      stage2_method=method)
    say({q: info[q] for q in ("status", "mv_total", "mv_stage1", "mv_stage2", "stage2_pairs")})
    assert info["status"] == 0 and info["mv_stage1"] == 0 and info["stage2_pairs"] == 3
    assert np.all(np.abs(sig - sigx[:3]) <= 1e-10 * sigx[:3])
    assert np.all(dense.triplet_residuals(A, sig, as_np(U), as_np(V)) <= 1e-12)
    out = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0, init_V=V0, shifts=shifts,
                    stage2_method=method)
    assert out["converged"]
    ratio = info["mv_total"] / out["stats"].mv_total
    say("MV gpu/oracle", ratio)
    assert 0.5 <= ratio <= 2.0


@gpu
def test_initial_basis_of_k0_vectors():
    """init_V without shifts: stage 1 starts from k0 given vectors."""
    need_gpu()
    import paper_1408_5535_amd as P
    N = 16
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    X0 = torch.tensor(np.random.default_rng(36).standard_normal((A.shape[1], 6)))
    sig, U, V, info = P.svds_smallest(to_dev(A), 6, 1e-12, block=2, anorm=an, init_V=X0)
    assert info["status"] == 0
    assert np.all(np.abs(sig - cf.grid_sigmas(N)[:6]) <= 1e-10 * cf.grid_sigmas(N)[:6])


def _scrambled_pair(sm_scale, seed=0, n=300):
    """A = Q1 diag(s) Q2^T (s: 1e-3, 2e-3, 3e-3, then linspace(0.01, 1)) and
    the dense M^-1 of M = Q1 diag(sm) Q2^T, sm = s with the given entries
    scaled."""
    rng = np.random.default_rng(seed)
    Q1 = np.linalg.qr(rng.standard_normal((n, n)))[0]
    Q2 = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.concatenate([[1e-3, 2e-3, 3e-3], np.linspace(0.01, 1, n - 3)])
    sm = s.copy()
    for j, f in sm_scale.items():
        sm[j] *= f
    A = Q1 @ np.diag(s) @ Q2.T
    return sp.csr_matrix(A), s, Q2 @ np.diag(1.0 / sm) @ Q1.T


@gpu
@pytest.mark.parametrize("method", ["gdk", "jdqmr"])
@pytest.mark.parametrize("mixed", [False, True])
def test_user_A_preconditioner_vs_oracle(method, mixed):
    """USER_A: solves with M ~ A (here M = A up to sigma_10 scaled by 2),
    formed by the library into M^-1 M^-T for C and [M^-1 g; M^-T f] for B
    (Section 4); float64, and a float32 first stage."""
    need_gpu()
    import paper_1408_5535_amd as P
    A, s, Mi = _scrambled_pair({10: 2.0})
    Mi_d = torch.tensor(Mi, device="cuda")
    calls = {"fp64": set(), "trans": set()}

    def solve(X, Y, trans, fp64):
        calls["fp64"].add(fp64)
        calls["trans"].add(trans)
        M = Mi_d.T if trans else Mi_d  # rows: X (b x rows_in) @ op(M)^T
        Y.copy_((X.double() @ M.T).to(Y.dtype))

    say("USER_A, scrambled n=300, method", method, "float32 stage 1", mixed)
    sig, U, V, info = P.svds_smallest(to_dev(A), 3, 1e-12, block=1, anorm=1.0,
                                      precond="user_A", user_solve=solve, stage2_method=method,
                                      stage1_fp32=mixed, fp64_continue=False, stage2="force")
    say({q: info[q] for q in ("status", "mv_total", "stage2_pairs", "iters1", "iters2")}, calls)
    assert info["status"] == 0 and info["stage2_pairs"] == 3
    assert calls["trans"] == {False, True}
    assert calls["fp64"] == ({False, True} if mixed else {True})
    assert np.all(np.abs(sig - s[:3]) <= 1e-10 * s[:3])
    assert np.all(dense.triplet_residuals(A, sig, as_np(U), as_np(V)) <= 1e-12)
    if not mixed:
        out = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0, stage2="force", stage2_method=method,
                        precond=("inverse_A", lambda Y: Mi @ Y, lambda X: Mi.T @ X))
        assert out["converged"]
        ratio = info["mv_total"] / out["stats"].mv_total
        say("MV gpu/oracle", ratio)
        assert 0.5 <= ratio <= 2.0


@gpu
@pytest.mark.parametrize("method", ["gdk", "jdqmr"])
def test_user_preconditioner_of_B_directly(method):
    """USER with user_apply_B only: no preconditioner in stage 1, the
    caller's M_B = [0 M^-1; M^-T 0] in stage 2 (also inside JDQMR)."""
    need_gpu()
    import paper_1408_5535_amd as P
    A, s, Mi = _scrambled_pair({10: 2.0})
    n = A.shape[1]
    Mi_d = torch.tensor(Mi, device="cuda")
    seen = []

    def applyB(R, T, theta, fp64):
        seen.append(len(theta))
        f, g = R[:, :n], R[:, n:]
        T[:, :n] = g @ Mi_d.T
        T[:, n:] = f @ Mi_d

    def MB(R, theta):
        return np.vstack([Mi @ R[n:], Mi.T @ R[:n]])

    say("USER direct B-preconditioner, method", method)
    sig, U, V, info = P.svds_smallest(to_dev(A), 3, 1e-12, block=1, anorm=1.0, precond="user",
                                      user_apply_B=applyB, stage2_method=method, stage2="force")
    say({q: info[q] for q in ("status", "mv_total", "stage2_pairs")}, len(seen))
    assert info["status"] == 0 and info["stage2_pairs"] == 3 and len(seen) > 0
    assert np.all(np.abs(sig - s[:3]) <= 1e-10 * s[:3])
    assert np.all(dense.triplet_residuals(A, sig, as_np(U), as_np(V)) <= 1e-12)
    out = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0, stage2="force", stage2_method=method,
                    precond=("B", MB))
    assert out["converged"]
    ratio = info["mv_total"] / out["stats"].mv_total
    say("MV gpu/oracle", ratio)
    assert 0.5 <= ratio <= 2.0


@gpu
def test_user_preconditioner_float64_continuation_gets_float64_blocks():
    """A float32 first stage continued in float64: the continuation calls
    the caller's M with float64 blocks (fp64 = 1)."""
    need_gpu()
    import paper_1408_5535_amd as P
    A, sigx, Ux, Vx = _givens_small()
    D = to_dev(A)
    d64 = torch.zeros(A.shape[1], dtype=torch.float64, device="cuda").index_add_(
        0, D.colind.long(), D.val * D.val)
    pairs = set()

    def apply(R, T, theta, fp64):
        pairs.add((R.dtype, fp64))
        T.copy_(R / (d64 if fp64 else d64.float())[None, :])

    sig, U, V, info = P.svds_smallest(D, 3, 1e-12, block=1, anorm=1.0, precond="user",
                                      user_apply=apply, stage1_fp32=True, fp64_continue=True)
    say(info["status"], pairs)
    assert info["status"] == 0
    assert pairs == {(torch.float32, False), (torch.float64, True)}
    assert np.all(np.abs(sig - sigx[:3]) <= 1e-10 * sigx[:3])


@gpu
@pytest.mark.parametrize("method", ["gdk", "jdqmr"])
def test_operator_for_A_matches_the_csr_path(method):
    """phsvds_svds_op: the products of the whole path through the caller's
    operator (here torch's dense float64 product) give the CSR path's
    triplets; sigma against the closed form."""
    need_gpu()
    import paper_1408_5535_amd as P
    A, sigx, Ux, Vx = _givens_small()
    Ad = torch.tensor(A.toarray(), device="cuda")
    calls = {"A": 0, "At": 0}

    def apply(X, Y, trans):
        calls["At" if trans else "A"] += 1
        Y.copy_((Ad.T if trans else Ad) @ X)

    say("operator for A, givens 240 x 200, method", method)
    op = P.Operator(A.shape[0], A.shape[1], apply)
    sig, U, V, info = P.svds_smallest(op, 3, 1e-12, block=1, anorm=1.0, stage2_method=method)
    say({q: info[q] for q in ("status", "mv_total", "stage2_pairs")}, calls)
    assert info["status"] == 0 and calls["A"] > 0 and calls["At"] > 0
    assert np.all(np.abs(sig - sigx[:3]) <= 1e-10 * sigx[:3])
    assert np.all(dense.triplet_residuals(A, sig, as_np(U), as_np(V)) <= 1e-12)
    sig2, _, _, info2 = P.svds_smallest(to_dev(A), 3, 1e-12, block=1, anorm=1.0,
                                        stage2_method=method)
    say("csr path", info2["mv_total"])
    assert np.all(np.abs(sig - sig2) <= 1e-12 * sig2)
    assert abs(info["mv_total"] - info2["mv_total"]) <= 0.2 * info2["mv_total"]


@gpu
def test_operator_largest_end_block_and_errors():
    need_gpu()
    import paper_1408_5535_amd as P
    N = 16
    A = wl.grid_gradient(N)
    An = torch.tensor(A.toarray(), device="cuda")

    def apply(X, Y, trans):
        Y.copy_((An.T if trans else An) @ X)

    op = P.Operator(A.shape[0], A.shape[1], apply)
    sig, U, V, info = P.svds_smallest(op, 4, 1e-12, block=4, which="largest",
                                      anorm=cf.grid_norm(N))
    ex = cf.grid_sigmas(N)[::-1][:4]
    assert info["status"] == 0 and np.all(np.abs(sig - ex) <= 1e-10 * ex)
    with pytest.raises(RuntimeError, match=r"\(-1\)"):
        P.svds_smallest(op, 2, 1e-10, precond="jacobi")
    with pytest.raises(RuntimeError, match=r"\(-1\)"):
        P.svds_smallest(op, 2, 1e-10, stage1_fp32=True)

    def bad(X, Y, trans):
        raise ValueError("no products today")

    with pytest.raises(RuntimeError, match=r"\(-5\)"):
        P.svds_smallest(P.Operator(A.shape[0], A.shape[1], bad), 2, 1e-10)


@gpu
@pytest.mark.parametrize("method", ["gdk", "jdqmr"])
def test_shift_invert_vs_oracle(method):
    """c_apply with c_inverse: the first stage on the caller's C^-1 (largest
    end), then the transition and the second stage on A; sigma against the
    closed form, products against the oracle's shift-invert."""
    need_gpu()
    import paper_1408_5535_amd as P
    A, sigx, Ux, Vx = _givens_small()
    Ci = (Vx / sigx ** 2) @ Vx.T
    Ci_d = torch.tensor(Ci, device="cuda")
    calls = []

    def cinv(X, Y):
        calls.append(X.shape[1])
        Y.copy_(Ci_d @ X)

    say("shift-invert, givens 240 x 200, method", method)
    sig, U, V, info = P.svds_smallest(to_dev(A), 3, 1e-12, block=1, anorm=1.0, c_apply=cinv,
                                      c_inverse=True, stage2_method=method)
    say({q: info[q] for q in ("status", "mv_total", "mv_stage1", "stage2_pairs")}, len(calls))
    assert info["status"] == 0 and info["stage2_pairs"] == 3 and len(calls) > 0
    assert np.all(np.abs(sig - sigx[:3]) <= 1e-10 * sigx[:3])
    assert np.all(dense.triplet_residuals(A, sig, as_np(U), as_np(V)) <= 1e-12)
    out = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0, c_apply=lambda X: Ci @ X, c_inverse=True,
                    stage2_method=method)
    assert out["converged"]
    ratio = info["mv_total"] / out["stats"].mv_total
    say("MV gpu/oracle", ratio, "stage 1", info["mv_stage1"], out["stats"].mv_stage1)
    assert 0.5 <= ratio <= 2.0


@gpu
def test_C_operator_and_shift_invert_grid():
    need_gpu()
    import paper_1408_5535_amd as P
    N = 16
    A = wl.grid_gradient(N)
    C = (A.T @ A).toarray()
    C_d = torch.tensor(C, device="cuda")
    Ci_d = torch.tensor(np.linalg.inv(C), device="cuda")
    ex = cf.grid_sigmas(N)[:4]
    # block 4 (with block 2 the first stage on C^-1 stalls on the double
    # pair sigma = 0.411 at 1.4e-12 relative, above the shift-invert test)
    for M, inv in ((C_d, False), (Ci_d, True)):
        sig, U, V, info = P.svds_smallest(to_dev(A), 4, 1e-12, block=4, anorm=cf.grid_norm(N),
                                          c_apply=lambda X, Y, M=M: Y.copy_(M @ X),
                                          c_inverse=inv)
        say("grid N=16 k=4, C operator, inverse", inv, info["status"], info["mv_stage1"])
        assert info["status"] == 0 and np.all(np.abs(sig - ex) <= 1e-10 * ex)
    with pytest.raises(RuntimeError, match=r"\(-1\)"):
        P.svds_smallest(to_dev(A), 4, 1e-12, c_apply=lambda X, Y: Y.copy_(X), c_inverse=True,
                        precond="jacobi")
