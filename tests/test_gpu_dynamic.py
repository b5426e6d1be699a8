"""Dynamic switching between C and B (Section 4.1, Algorithm 3) on the GPU
through the C ABI, against the CPU oracle's switching (oracle.dynamic) and
the stated spectra.

* Scrambled 300 x 300 matrices with M ~ A given by its solves (USER_A):
  M = A (C locks all three pairs in the first run) and M = A up to one
  singular value scaled by 1e-9 (C stalls, the first B run locks all
  three): the same runs and choice as the oracle, sigma to 1e-10, residuals
  to 1e-12 ||A||, products within a factor 2 of the oracle's.
* A 240 x 200 Givens-scrambled matrix (sigma_1..3 = 1e-4, 2e-4, 3e-4) with
  no preconditioner and with Jacobi: rates of the two approaches lie close,
  so the later runs may differ from the oracle's by rounding; the first two
  runs, the result and the residuals are checked."""
import numpy as np
import pytest
import torch

from oracle import dense, dynamic as dy
from tests.gpu_util import as_np, gpu, need_gpu, say, to_dev
from tests.test_gpu_boundary import _givens_small, _scrambled_pair


@gpu
@pytest.mark.parametrize("case", ["good", "mismatch"])
def test_dynamic_scrambled_user_A_vs_oracle(case):
    need_gpu()
    import paper_1408_5535_amd as P
    A, s, Mi = _scrambled_pair({150: 1e-9} if case == "mismatch" else {})
    Mi_d = torch.tensor(Mi, device="cuda")

    def solve(X, Y, trans, fp64):
        M = Mi_d.T if trans else Mi_d
        Y.copy_((X.double() @ M.T).to(Y.dtype))

    say("dynamic switching, scrambled n=300, M case", case)
    sig, U, V, info = P.svds_smallest(to_dev(A), 3, 1e-12, block=1, anorm=1.0,
                                      precond="user_A", user_solve=solve, dynamic=True,
                                      stage2_method="gdk")
    dyn = info["dynamic"]
    say({q: info[q] for q in ("status", "mv_total", "stage2_pairs")}, dyn)
    out = dy.phsvds_dynamic(A, 3, 1e-12, precond=("inverse_A", lambda Y: Mi @ Y,
                                                  lambda X: Mi.T @ X),
                            anorm=1.0, stage2_method="gdk")
    say("oracle", out["dynamic"], out["stats"].mv_total)
    assert info["status"] == 0
    assert (dyn["choice"], dyn["how"]) == (out["dynamic"]["choice"], out["dynamic"]["how"])
    assert [(r[0], r[1], r[3]) for r in dyn["runs"]] == \
        [(r[0], r[1], r[3]) for r in out["dynamic"]["runs"]]
    assert np.all(np.abs(sig - s[:3]) <= 1e-10 * s[:3])
    assert np.all(dense.triplet_residuals(A, sig, as_np(U), as_np(V)) <= 1e-12)
    ratio = info["mv_total"] / out["stats"].mv_total
    say("MV gpu/oracle", ratio)
    assert 0.5 <= ratio <= 2.0


@gpu
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_dynamic_givens_closed_form(precond):
    need_gpu()
    import paper_1408_5535_amd as P
    A, sigx, Ux, Vx = _givens_small()
    say("dynamic switching, givens 240 x 200, precond", precond)
    sig, U, V, info = P.svds_smallest(to_dev(A), 3, 1e-12, block=1, anorm=1.0,
                                      precond=precond, dynamic=True, stage2_method="gdk")
    dyn = info["dynamic"]
    say({q: info[q] for q in ("status", "mv_total", "stage2_pairs")}, dyn)
    assert info["status"] == 0
    assert [(r[0], r[1]) for r in dyn["runs"][:2]] == [("C", 50), ("B", 50)]
    assert np.all(np.abs(sig - sigx[:3]) <= 1e-10 * sigx[:3])
    assert np.all(dense.triplet_residuals(A, sig, as_np(U), as_np(V)) <= 1e-12)


@gpu
def test_dynamic_rejects_unsupported_settings():
    need_gpu()
    import paper_1408_5535_amd as P
    A, sigx, Ux, Vx = _givens_small()
    D = to_dev(A)
    for kw in ({"stage1_fp32": True}, {"stage2_method": "jdqmr"}, {"which": "largest"}):
        with pytest.raises(RuntimeError, match=r"\(-1\)"):
            P.svds_smallest(D, 3, 1e-12, dynamic=True, **{"stage2_method": "gdk", **kw})
