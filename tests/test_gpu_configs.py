"""Members of the benchmark families at their stated spectra, on the GPU
through the C ABI against the CPU oracle run with the same readings.

* The log-spaced Givens matrix (1200 x 1000, sigma = logspace(-4, 0), 3n
  rotations each side, k = 5, block 1, no preconditioner): its smallest
  gaps in C are ~1e-10 of ||C||, beyond any unpreconditioned budget; both
  solvers stop at the same product budget, report not converged, and their
  best Ritz values bound the exact ones from above.
* A reduced weighted grid (N = 64, rows scaled by lognormal(0, 1) weights,
  k = 16, block 8, Jacobi): float64 and float32-first-stage solves against
  the float64 oracle, per triplet."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla
import torch

import workloads as wl
from oracle import dense, phsvds as ph
from tests.gpu_util import as_np, gpu, need_gpu, say, to_dev


@gpu
def test_givens_logspaced_stated_spectrum_under_a_budget():
    need_gpu()
    import paper_1408_5535_amd as P
    A, sig, U, V = wl.givens_scrambled(seed=1)  # m 1200, n 1000, 3n rotations
    say("givens log-spaced, nnz", A.nnz, "k=5 b=1, 20000 products")
    X0 = torch.tensor(wl.initial_block(A.shape[1], 1, 2))
    s_gpu, Ug, Vg, info = P.svds_smallest(to_dev(A), 5, 1e-12, block=1, anorm=1.0,
                                          init_block=X0, max_matvecs=20000)
    say({q: info[q] for q in ("status", "mv_total", "iters1")}, s_gpu, info["res"])
    assert info["status"] == 1
    out = ph.phsvds(A, 5, 1e-12, block=1, anorm=1.0, max_iters=20000)
    say("oracle", out["sigma"], out["res"])
    assert not out["converged"]
    for s_best in (s_gpu, out["sigma"]):
        # Ritz values of C bound the exact eigenvalues from above
        assert np.all(s_best >= sig[:5] * (1 - 1e-12))
    assert np.max(info["res"]) > 1e-12 and np.max(out["res"]) > 1e-12
    res = dense.triplet_residuals(A, s_gpu, as_np(Ug), as_np(Vg))
    assert np.allclose(res, info["res"], rtol=1e-6)


@gpu
def test_reduced_weighted_grid_vs_oracle():
    need_gpu()
    import paper_1408_5535_amd as P
    N, k, b = 64, 16, 8
    A = wl.grid_gradient(N, weights="lognormal", seed=3)
    an = float(sla.svds(A, k=1, which="LM", return_singular_vectors=False, tol=1e-12)[0])
    out = ph.phsvds(A, k, 1e-12, block=b, anorm=an, precond="jacobi")
    assert out["converged"]
    sig_ref = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:k]
    assert np.allclose(out["sigma"], sig_ref, rtol=1e-10, atol=0)
    X0 = torch.tensor(wl.initial_block(A.shape[1], b, 2))
    for mixed in (False, True):
        say("weighted grid N=64 k=16 b=8 Jacobi, float32 stage 1:", mixed)
        sig, U, V, info = P.svds_smallest(to_dev(A), k, 1e-12, block=b, anorm=an,
                                          precond="jacobi", init_block=X0, stage1_fp32=mixed)
        say({q: info[q] for q in ("status", "mv_total", "stage2_pairs", "fp32_locked")})
        assert info["status"] == 0
        assert np.all(np.abs(sig - out["sigma"]) <= 1e-10 * out["sigma"])
        res = dense.triplet_residuals(A, sig, as_np(U), as_np(V))
        assert np.all(res <= 1e-12 * an)
        if not mixed:
            ratio = info["mv_total"] / out["stats"].mv_total
            say("MV gpu/oracle", ratio)
            assert 0.5 <= ratio <= 2.0
