"""Pins of the oracle's operator forms (Section 3.3: A, or C, given as
functions) and of shift-invert (Section 4: the caller's C^-1), against
closed forms.

* Shift-invert on a grid (N = 16, k = 4, block 2) with C^-1 as a dense
  inverse: sigma to 1e-10 of the closed form, no second stage needed.
* Shift-invert on a 240 x 200 Givens-scrambled matrix with sigma_1..3 =
  1e-4..3e-4 and C^-1 = V diag(sigma^-2) V^T: ten or so products with C^-1
  lock the three pairs at C's accuracy floor, and the second stage takes
  them to 1e-12 ||A|| (without the inverse stage 1 needs hundreds).
* The first stage's test mapped onto C^-1 is exactly the test on C: for a
  pair of C with residual r_C, r' = C^-1 x - mu x satisfies C r' = -mu r_C.
* A given operator for C reproduces the CSR path."""
import numpy as np

import workloads as wl
from oracle import dense, phsvds as ph
from tests import closed_forms as cf


def test_shift_invert_grid_closed_form():
    N = 16
    A = wl.grid_gradient(N)
    Ci = np.linalg.inv((A.T @ A).toarray())
    out = ph.phsvds(A, 4, 1e-12, block=2, anorm=cf.grid_norm(N), c_apply=lambda X: Ci @ X,
                    c_inverse=True)
    ex = cf.grid_sigmas(N)[:4]
    assert out["converged"] and out["stats"].stage2_pairs == 0
    assert np.all(np.abs(out["sigma"] - ex) <= 1e-10 * ex)


def _givens():
    n, m = 200, 240
    s = np.concatenate([[1e-4, 2e-4, 3e-4], np.linspace(0.05, 1.0, n - 3)])
    return wl.givens_scrambled(m, n, s, rot_left=int(0.7 * m), rot_right=int(0.7 * n), seed=2)


def test_shift_invert_then_stage2_on_tiny_sigma():
    A, sx, U, V = _givens()
    Ci = (V / sx ** 2) @ V.T
    out = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0, c_apply=lambda X: Ci @ X, c_inverse=True)
    assert out["converged"] and out["stats"].stage2_pairs == 3
    assert out["stats"].mv_stage1 <= 30
    assert np.all(np.abs(out["sigma"] - sx[:3]) <= 1e-10 * sx[:3])
    assert np.all(dense.triplet_residuals(A, out["sigma"], out["U"], out["V"]) <= 1e-12)
    plain = ph.phsvds(A, 3, 1e-12, block=1, anorm=1.0)
    assert plain["stats"].mv_stage1 > 10 * out["stats"].mv_stage1


def test_inverse_residual_identity():
    A, sx, U, V = _givens()
    C = (A.T @ A).toarray()
    Ci = (V / sx ** 2) @ V.T
    x = V[:, 0] + 1e-3 * np.random.default_rng(4).standard_normal(V.shape[0])
    x /= np.linalg.norm(x)
    theta = float(x @ C @ x)
    mu = 1.0 / theta
    r_C = C @ x - theta * x
    r_inv = Ci @ x - mu * x
    assert np.linalg.norm(C @ r_inv + mu * r_C) <= 1e-9 * np.linalg.norm(mu * r_C)


def test_C_operator_reproduces_the_csr_path():
    N = 16
    A = wl.grid_gradient(N)
    C = (A.T @ A).toarray()
    a = ph.phsvds(A, 4, 1e-12, block=2, anorm=cf.grid_norm(N), c_apply=lambda X: C @ X)
    b = ph.phsvds(A, 4, 1e-12, block=2, anorm=cf.grid_norm(N))
    assert a["converged"] and b["converged"]
    assert np.all(np.abs(a["sigma"] - b["sigma"]) <= 1e-12 * b["sigma"])
    assert abs(a["stats"].mv_total - b["stats"].mv_total) <= 0.1 * b["stats"].mv_total
