"""Full PHSVDS on the GPU through the C ABI vs the CPU oracle and closed forms.

Bars: sigma within 1e-10 relative of the float64 oracle / closed form,
explicit float64 residual sqrt(||r_u||^2 + ||r_v||^2) <= 1e-12 ||A||, and
singular subspaces of complete clusters within 1e-8."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dense, phsvds as ph
from tests import closed_forms as cf
from tests.gpu_util import as_np, gpu, need_gpu, say, to_dev


def _solve(A, k, tol=1e-12, b=1, **kw):
    import paper_1408_5535_amd as P
    X0 = torch.tensor(wl.initial_block(A.shape[1], b, 2))
    return P.svds_smallest(to_dev(A), k, tol, block=b, init_block=X0, **kw)


def _check(A, sig, U, V, info, exact, anorm, tol=1e-12):
    U, V = as_np(U), as_np(V)
    assert info["status"] == 0, info
    assert np.all(np.abs(sig - exact) <= 1e-10 * exact), (sig, exact)
    res = dense.triplet_residuals(A, sig, U, V)
    assert np.all(res <= tol * anorm), res
    assert np.allclose(res, info["res"], rtol=1e-6, atol=1e-3 * tol * anorm)
    assert np.linalg.norm(V.T @ V - np.eye(len(sig))) < 1e-10
    return U, V


@gpu
def test_grid_smallest_closed_form_and_oracle():
    need_gpu()
    N = 16
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    say("grid smallest N=16 k=10 b=4")
    sig, U, V, info = _solve(A, 10, b=4, anorm=an)
    say(info)
    U, V = _check(A, sig, U, V, info, cf.grid_sigmas(N)[:10], an)
    out = ph.phsvds(A, 10, 1e-12, block=4, anorm=an)
    assert np.allclose(sig, out["sigma"], rtol=1e-10, atol=0)
    for g in cf.clusters(cf.grid_sigmas(N)[:10]):
        if g[-1] == 9:
            continue
        assert cf.principal_angles(V[:, g], out["V"][:, g]) < 1e-8
    ratio = info["mv_total"] / out["stats"].mv_total
    say("MV gpu/oracle", ratio)
    assert 0.5 <= ratio <= 2.0


@gpu
def test_grid_largest_closed_form():
    need_gpu()
    N = 16
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    say("grid largest N=16 k=10 b=4")
    sig, U, V, info = _solve(A, 10, b=4, anorm=an, which="largest")
    say(info)
    _check(A, sig, U, V, info, cf.grid_sigmas(N)[::-1][:10], an)
    assert info["stage2_pairs"] == 0


@gpu
@pytest.mark.parametrize("which", ["smallest", "largest"])
def test_grid_n128_both_ends_closed_form(which):
    """N = 128 (m = 33024, n = 16384), k = 10, block 4: the clustered
    largest end (relative gap 4e-5 after the 10th value) needs an accurate
    basis; sigma and residuals are checked against the closed form."""
    need_gpu()
    import paper_1408_5535_amd as P
    N = 128
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    say("grid N=128 k=10 b=4", which)
    sig, U, V, info = P.svds_smallest(to_dev(A), 10, 1e-12, block=4, which=which, anorm=an,
                                      max_matvecs=60000)
    say(info["mv_total"], info["status"])
    ex = cf.grid_sigmas(N)
    _check(A, sig, U, V, info, ex[:10] if which == "smallest" else ex[::-1][:10], an)


@gpu
@pytest.mark.parametrize("b", [3, 8])
def test_grid_block_widths_without_fused_gram(b):
    """Block widths whose CholQR Grams take the separate X^T X pass (3, 8)
    and whose X S products use the 4- and 8-column tiles: N = 24 grid,
    k = 8 smallest, sigma against the closed form, float64 residuals."""
    need_gpu()
    N = 24
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    say("grid N=24 k=8 b", b)
    sig, U, V, info = _solve(A, 8, b=b, anorm=an)
    say({k: info[k] for k in ("status", "mv_total", "iters1", "rollbacks1")
         if k in info})
    _check(A, sig, U, V, info, cf.grid_sigmas(N)[:8], an)


@gpu
def test_grid_n512_benchmark_configuration():
    """The benchmark's solve at full size: N = 512 (m = 525312, n = 262144),
    k = 10 smallest, block 4, float64, the paper's start block; sigma
    against the closed form and float64 residuals recomputed on the host."""
    need_gpu()
    import paper_1408_5535_amd as P
    N = 512
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    say("grid N=512 k=10 b=4 (benchmark configuration)")
    sig, U, V, info = P.svds_smallest(to_dev(A), 10, 1e-12, block=4)
    say({k: info[k] for k in ("status", "mv_total", "iters1", "stage2_pairs")})
    _check(A, sig, U, V, info, cf.grid_sigmas(N)[:10], an)
    assert info["stage2_pairs"] == 0


@gpu
def test_givens_two_stage_closed_form():
    need_gpu()
    n, m = 200, 240
    s = np.concatenate([[1e-3, 2e-3, 3e-3, 4e-3, 5e-3], np.linspace(0.05, 1.0, n - 5)])
    A, sigx, Ux, Vx = wl.givens_scrambled(m, n, s, rot_left=int(0.7 * m), rot_right=int(0.7 * n),
                                          seed=1)
    say("givens two-stage n=200 k=5 b=1")
    sig, U, V, info = _solve(A, 5, b=1, anorm=1.0)
    say(info)
    assert info["stage2_pairs"] >= 1
    U, V = _check(A, sig, U, V, info, sigx[:5], 1.0)
    for i in range(5):
        assert abs(abs(V[:, i] @ Vx[:, i]) - 1) < 1e-12
        assert abs(abs(U[:, i] @ Ux[:, i]) - 1) < 1e-12


@gpu
def test_forced_stage2_grid():
    need_gpu()
    N = 16
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    say("grid forced stage 2 k=6 b=2")
    sig, U, V, info = _solve(A, 6, b=2, anorm=an, stage2="force")
    say(info)
    assert info["stage2_pairs"] == 6
    _check(A, sig, U, V, info, cf.grid_sigmas(N)[:6], an)


@gpu
def test_mixed_precision_weighted_grid_vs_oracle():
    """Float32 stage 1 (with and without the float64 continuation) then
    float64 stage 2, per triplet against the float64 oracle's two-stage
    result: sigma within 1e-10 relative, and the sine of the angle between
    the right singular vectors within max(1e-8, 4 r / gap), r the float64
    residual bound and gap the distance to the nearest other singular value
    (the sin-theta bound)."""
    need_gpu()
    N = 24
    A = wl.grid_gradient(N, weights="lognormal", seed=3)
    an = float(np.linalg.norm(A.toarray(), 2))
    k = 6
    sig_all = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))
    sig_ex = sig_all[:k]
    gap = np.array([np.min(np.abs(np.delete(sig_all, i) - sig_all[i])) for i in range(k)])
    out = ph.phsvds(A, k, 1e-12, block=4, anorm=an)
    assert np.allclose(out["sigma"], sig_ex, rtol=1e-10, atol=0)
    say("mixed precision weighted grid N=24 k=6 b=4")
    for cont in (True, False):
        sig, U, V, info = _solve(A, k, b=4, anorm=an, stage1_fp32=True, fp64_continue=cont)
        say(cont, info)
        U, V = _check(A, sig, U, V, info, sig_ex, an)
        for i in range(k):
            err = abs(sig[i] - out["sigma"][i]) / out["sigma"][i]
            ang = cf.principal_angles(V[:, [i]], out["V"][:, [i]])
            say(f"  continue={cont} triplet {i}: sigma {sig[i]:.15e}, rel. error vs the "
                f"float64 oracle {err:.1e}, sin angle {ang:.1e} (gap {gap[i]:.1e})")
            assert err <= 1e-10
            assert ang <= max(1e-8, 4 * 1e-12 * an / gap[i])


@gpu
def test_jacobi_random_sparse_vs_dense_definition():
    need_gpu()
    A = wl.random_sparse(300, 200, 8, seed=21)
    sigx, Ux, Vx = dense.svd_extreme_dense(A, 4)
    an = float(np.linalg.norm(A.toarray(), 2))
    say("jacobi random sparse 300x200 k=4 b=2")
    sig, U, V, info = _solve(A, 4, b=2, anorm=an, precond="jacobi")
    say(info)
    U, V = _check(A, sig, U, V, info, sigx, an)
    for i in range(4):
        assert abs(abs(V[:, i] @ Vx[:, i]) - 1) < 1e-10


@gpu
@pytest.mark.parametrize("mixed", [False, True])
def test_out_of_budget_returns_best_approximations(mixed):
    """A solve stopped by its product budget returns status 1 with every
    triplet filled: the unlocked pairs are the current Ritz approximations,
    each with its true float64 residual, and a Ritz value of C bounds the
    smallest singular value from above."""
    need_gpu()
    N = 32
    A = wl.grid_gradient(N)
    an = cf.grid_norm(N)
    k = 6
    say(f"grid N={N} k={k} b=2 max_matvecs=40 mixed={mixed}")
    sig, U, V, info = _solve(A, k, b=2, anorm=an, max_matvecs=40, stage1_fp32=mixed)
    say(info)
    U, V = as_np(U), as_np(V)
    assert info["status"] == 1
    assert np.all(np.isfinite(sig)) and np.all(np.isfinite(info["res"]))
    assert np.all(np.diff(sig) >= 0)
    res = dense.triplet_residuals(A, sig, U, V)
    assert np.allclose(res, info["res"], rtol=1e-6, atol=1e-14 * an)
    assert np.max(res) > 1e-12 * an
    assert np.allclose(np.linalg.norm(U, axis=0), 1.0, atol=1e-12)
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-12)
    assert sig[0] >= cf.grid_sigmas(N)[0] * (1 - 1e-12)
