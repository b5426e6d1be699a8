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
