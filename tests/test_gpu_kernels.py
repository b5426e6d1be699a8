"""GPU kernels through the C ABI vs plain definitions (scipy products)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as wl
from tests.gpu_util import as_np, gpu, need_gpu, say, to_dev


def _mats():
    r = np.random.default_rng(7)
    out = {"grid16": wl.grid_gradient(16), "rand": wl.random_sparse(3000, 2000, 12, seed=3)}
    # empty rows, one 2000-entry row, power-law rows
    B = sp.random(4000, 2500, density=0.002, format="lil", random_state=1)
    B[5, :] = 0
    B[17, :2000] = r.standard_normal(2000)
    out["ragged"] = sp.csr_matrix(B)
    out["powerlaw"] = wl.powerlaw_sparse(20000, 15000, mean=10, kmax=2000, seed=4)
    return out


@gpu
@pytest.mark.parametrize("name", ["grid16", "rand", "ragged", "powerlaw"])
@pytest.mark.parametrize("b", [1, 4, 8, 32])
def test_spmm_f64_matches_scipy(name, b):
    need_gpu()
    import paper_1408_5535_amd as P
    A = _mats()[name]
    say("spmm f64", name, A.shape, A.nnz, "b", b)
    X = np.random.default_rng(b).standard_normal((A.shape[1], b))
    Ad = to_dev(A)
    Y = as_np(P.spmm(Ad, torch.tensor(X, device="cuda")))
    ref = A @ X
    scale = abs(A) @ abs(X)
    assert np.all(np.abs(Y - ref) <= 1e-14 * scale + 1e-300)
    Ya = as_np(P.spmm(Ad, torch.tensor(X, device="cuda"), absval=True))
    assert np.allclose(Ya, scale, rtol=1e-14, atol=0)


@gpu
@pytest.mark.parametrize("name", ["grid16", "powerlaw"])
def test_spmm_f32_matches_scipy(name):
    need_gpu()
    import paper_1408_5535_amd as P
    A = _mats()[name]
    say("spmm f32", name)
    X = np.random.default_rng(1).standard_normal((A.shape[1], 8)).astype(np.float32)
    Ad = to_dev(A)
    Y = as_np(P.spmm(Ad, torch.tensor(X, device="cuda")))
    A32 = A.astype(np.float32).astype(np.float64)
    ref = A32 @ X.astype(np.float64)
    scale = abs(A32) @ abs(X.astype(np.float64))
    assert np.all(np.abs(Y - ref) <= 4e-6 * scale + 1e-30)


@gpu
@pytest.mark.parametrize("name", ["grid16", "rand", "ragged", "powerlaw"])
def test_csr_transpose_exact(name):
    need_gpu()
    import paper_1408_5535_amd as P
    A = _mats()[name]
    say("transpose", name)
    At = P.csr_transpose(to_dev(A))
    ref = A.T.tocsr()
    ref.sort_indices()
    assert np.array_equal(as_np(At.rowptr), ref.indptr)
    assert np.array_equal(as_np(At.colind), ref.indices)
    assert np.array_equal(as_np(At.val), ref.data)


def _rr_cases():
    r = np.random.default_rng(11)
    out = []
    for p in (1, 2, 7, 35, 64):
        X = r.standard_normal((p, p))
        out.append((f"random{p}", X + X.T))
    Q, _ = np.linalg.qr(r.standard_normal((40, 40)))
    spectra = {
        "clustered": np.r_[1e-4 + 1e-6 * np.arange(1, 21), np.linspace(0.1, 8, 20)],
        "repeated": np.r_[np.ones(10), 2 * np.ones(10), np.linspace(3, 4, 20)],
        "graded": np.logspace(-12, 0, 40),
        "identity": np.ones(40),
        "zero": np.zeros(40),
    }
    for name, ev in spectra.items():
        out.append((name, Q @ np.diag(ev) @ Q.T))
    out.append(("diagonal", np.diag(np.arange(40.0))))
    W = np.diag(np.abs(np.arange(-10, 11)).astype(float)) + np.diag(np.ones(20), 1) + \
        np.diag(np.ones(20), -1)
    out.append(("wilkinson21", W))
    return out


@gpu
@pytest.mark.parametrize("case", range(12))
def test_rr_eig_selected_pairs(case):
    """Selected eigenpairs of the Rayleigh-Ritz matrix: eigenvalues against
    LAPACK (numpy eigvalsh), residual and orthonormality of the vectors."""
    need_gpu()
    import paper_1408_5535_amd as P
    name, H = _rr_cases()[case]
    p = H.shape[0]
    nrm = np.linalg.norm(H, 2)
    ref = np.linalg.eigvalsh(H)
    for nvec in sorted({1, min(4, p), min(24, p), p}):
        for largest in (False, True):
            say("rr_eig", name, "p", p, "nvec", nvec, "largest", largest)
            th, S = P.rr_eig(torch.tensor(H, device="cuda"), nvec, largest)
            th, S = as_np(th), as_np(S)
            want = ref[::-1] if largest else ref
            got = np.r_[th[:nvec], th[p - 1]]
            exp = np.r_[want[:nvec], want[p - 1]]
            assert np.max(np.abs(got - exp)) <= 1e-14 * nrm + 1e-30, (name, nvec, largest)
            Sv = S[:, :nvec]
            res = np.linalg.norm(H @ Sv - Sv * th[:nvec], axis=0)
            assert np.max(res) <= 1e-14 * nrm + 1e-30, (name, nvec, largest)
            assert np.max(np.abs(Sv.T @ Sv - np.eye(nvec))) <= 1e-13, (name, nvec, largest)


_FULL = {}


def _full(family):
    """Full-size matrices of the benchmark families (built once per session)."""
    if family not in _FULL:
        if family == "weighted1024":
            _FULL[family] = wl.grid_gradient(1024, weights="lognormal", seed=3)
        else:
            _FULL[family] = wl.powerlaw_sparse()
    return _FULL[family]


@gpu
@pytest.mark.parametrize("family", ["weighted1024", "powerlaw"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_spmm_full_size_sampled_rows(family, dtype):
    """A X and A^T Y at the full sizes of the weighted N=1024 grid
    (2099200 x 1048576) and the power-law matrix (4M x 3M, rows up to 2000
    entries), block 8, with the launch configuration the solver uses;
    sampled rows (seeded, plus the longest row and both ends) against SciPy
    in float64 within the forward-error bound (len + 2) u sum |a||x|."""
    need_gpu()
    import paper_1408_5535_amd as P
    A = _full(family)
    m, n = A.shape
    b = 8
    say("spmm full size", family, dtype, A.shape, A.nnz)
    r = np.random.default_rng(5)
    X = r.standard_normal((n, b))
    Ad = to_dev(A)
    At = P.csr_transpose(Ad)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    Aref = A if dtype == "f64" else A.astype(np.float32).astype(np.float64)
    Xd = torch.tensor(X, dtype=tdt, device="cuda")
    Xref = X if dtype == "f64" else X.astype(np.float32).astype(np.float64)
    Y = P.spmm(Ad, Xd)
    lens = np.diff(A.indptr)
    rows = np.unique(np.r_[r.choice(m, 4096, replace=False), np.argmax(lens), 0, m - 1])
    Yh = as_np(Y[torch.tensor(rows, device="cuda")]).astype(np.float64)
    ref = Aref[rows] @ Xref
    bound = (lens[rows] + 2)[:, None] * u * (abs(Aref[rows]) @ abs(Xref)) + 1e-300
    assert np.all(np.abs(Yh - ref) <= bound)
    # A^T Y through the device transpose: columns of A are the rows of A^T
    Yfull = Y.double().cpu().numpy()
    Yin = Yfull if dtype == "f64" else Yfull.astype(np.float32).astype(np.float64)
    Z = P.spmm(At, torch.tensor(Yin, dtype=tdt, device="cuda"))
    cl = np.bincount(A.indices, minlength=n)
    cols = np.unique(np.r_[r.choice(n, 4096, replace=False), np.argmax(cl), 0, n - 1])
    Zh = as_np(Z[torch.tensor(cols, device="cuda")]).astype(np.float64)
    AcT = Aref.tocsc()[:, cols].T.tocsr()
    zref = AcT @ Yin
    zb = (cl[cols] + 2)[:, None] * u * (abs(AcT) @ abs(Yin)) + 1e-300
    assert np.all(np.abs(Zh - zref) <= zb)


def _svd_cases():
    r = np.random.default_rng(11)
    out = [("random 20x10", r.standard_normal((20, 10))),
           ("square 64", r.standard_normal((64, 64))),
           ("128x64", r.standard_normal((128, 64))),
           ("odd 33x7", r.standard_normal((33, 7))),
           ("1x1", np.array([[-3.0]]))]
    # two equal columns: a zero singular value
    M = r.standard_normal((16, 8))
    M[:, 5] = M[:, 2]
    out.append(("rank-deficient", M))
    # singular value 1 of multiplicity three
    Q1, _ = np.linalg.qr(r.standard_normal((30, 12)))
    Q2, _ = np.linalg.qr(r.standard_normal((12, 12)))
    out.append(("repeated", (Q1 * np.r_[1.0, 1.0, 1.0, np.linspace(0.1, 0.9, 9)]) @ Q2.T))
    # column-graded: well-conditioned B times diag(1 .. 1e-12)
    out.append(("graded", r.standard_normal((40, 12)) * np.logspace(0, -12, 12)))
    return out


@gpu
@pytest.mark.parametrize("case", range(8))
def test_small_svd_vs_lapack_and_jacobi(case):
    """The refined projection's small SVD (one-sided Jacobi on the GPU):
    singular values against LAPACK (numpy) within 1e-14 sigma_max; for the
    column-graded case against the oracle's float64 one-sided Jacobi within
    1e-12 relative, since there LAPACK's absolute accuracy says nothing of
    the small values; right vectors orthonormal and ||M y_j|| = sigma_j."""
    need_gpu()
    import paper_1408_5535_amd as P
    from oracle.dense import jacobi_svd
    name, M = _svd_cases()[case]
    rows, cols = M.shape
    say("small_svd", name, rows, "x", cols)
    sv, Y = P.small_svd(torch.tensor(M, device="cuda"))
    sv, Y = as_np(sv), as_np(Y)
    smax = np.linalg.norm(M, 2)
    assert np.all(np.diff(sv) >= 0), sv
    ref = np.sort(np.linalg.svd(M, compute_uv=False))
    assert np.max(np.abs(sv - ref)) <= 1e-14 * smax + 1e-300, (name, sv, ref)
    if name == "graded":
        _, sj, _ = jacobi_svd(M)
        sj = np.sort(sj)
        assert np.all(np.abs(sv - sj) <= 1e-12 * sj), (sv, sj)
    assert np.max(np.abs(Y.T @ Y - np.eye(cols))) <= 1e-13, name
    got = np.linalg.norm(M @ Y, axis=0)
    assert np.all(np.abs(got - sv) <= 1e-14 * smax + 1e-12 * sv), (name, got, sv)


@gpu
def test_small_svd_rejects_sizes_out_of_range():
    need_gpu()
    import paper_1408_5535_amd as P
    for shape in ((10, 20), (200, 10), (70, 65)):
        with pytest.raises(RuntimeError):
            P.small_svd(torch.zeros(shape, dtype=torch.float64, device="cuda"))
