"""Pins of the oracle's preconditioner forms from M ~ A (Section 4) and of
its dynamic switching between C and B (Section 4.1, Algorithm 3).

* With M = A (square, nonsingular) the two forms are exactly C^-1 and B^-1.
* The harmonic Ritz extraction for the target 0 reproduces the eigenpairs
  of B on an invariant subspace and takes the smallest positive one.
* Algorithm 3's control loop against hand-traced run sequences: the first
  tests on C then B, maxIter doubling when the same approach wins and
  halving (floor(j / 2)) when it changes, the numConverged rules, the switch
  limit, and a run that locks every pair.
* End to end: the Section 5.1 switching matrix with its preconditioner
  M = A + diag(rand * 1e4), and scrambled matrices whose M fails on C but
  not on B, against the stated spectra."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dense, dynamic as dy, phsvds as ph


def _square(n=30, seed=5):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + n ** 0.5 * np.eye(n)


def test_M_equal_A_forms_are_the_exact_inverses():
    A = _square()
    n = A.shape[0]
    Ai = np.linalg.inv(A)
    pc1, pcB = ph.approx_A_forms(lambda Y: Ai @ Y, lambda X: Ai.T @ X, n)
    R = np.random.default_rng(6).standard_normal((n, 3))
    assert np.allclose(pc1(R, None, None), np.linalg.solve(A.T @ A, R), rtol=1e-10, atol=1e-12)
    B = np.block([[np.zeros((n, n)), A.T], [A, np.zeros((n, n))]])
    RB = np.random.default_rng(7).standard_normal((2 * n, 3))
    assert np.allclose(pcB(RB, None, None), np.linalg.solve(B, RB), rtol=1e-10, atol=1e-12)


def test_harmonic_zero_extraction_on_an_invariant_subspace():
    """V spans [v_i; +-u_i] for sigma = 0.5, 2, 3 of a 9 x 6 matrix, turned
    by a 1e-3 perturbation: the first candidate is sigma_1 = 0.5's positive
    pair (balanced, Rayleigh quotient 0.5 to the perturbation's square),
    ahead of -0.5 (negative) and the larger pairs."""
    m, n = 9, 6
    sig = np.array([0.5, 2.0, 3.0, 4.0, 5.0, 6.0])
    A, _, U, Vr = wl.givens_scrambled(m, n, sig, rot_left=30, rot_right=30, seed=3)
    A = A.toarray()
    cols = []
    for i in range(3):
        for sgn in (1.0, -1.0):
            cols.append(np.concatenate([Vr[:, i], sgn * U[:, i]]) / math.sqrt(2))
    V = np.linalg.qr(np.column_stack(cols) + 1e-3 * np.random.default_rng(8).standard_normal(
        (m + n, len(cols))))[0]
    B = np.block([[np.zeros((n, n)), A.T], [A, np.zeros((m, m))]])
    W = B @ V
    H = V.T @ W
    Y, lead = ph._harmonic0(V, W, H, n)
    x = V @ Y[:, 0]
    theta = float(Y[:, 0] @ H @ Y[:, 0])
    assert abs(2 * float(x[:n] @ x[:n]) - 1.0) < 0.1
    assert abs(theta - 0.5) < 1e-4 and abs(lead - 0.5) < 1e-2
    assert np.linalg.norm(B @ x - theta * x) < 6 * 1e-2  # ||B|| times the turn
    # the exact subspace gives the exact pair
    V0 = np.linalg.qr(np.column_stack(cols))[0]
    Y0, lead0 = ph._harmonic0(V0, B @ V0, V0.T @ B @ V0, n)
    x0 = V0 @ Y0[:, 0]
    assert abs(lead0 - 0.5) < 1e-13
    assert np.linalg.norm(B @ x0 - 0.5 * x0) < 1e-13


def _scripted(results):
    log = []
    it = iter(results)

    def run(ap, max_iter):
        want_ap, rate, locked = next(it)
        assert ap == want_ap, (ap, want_ap, log)
        log.append((ap, max_iter))
        return rate, locked
    return run, log


def test_switch_control_doubles_halves_and_decides():
    run, log = _scripted([("C", 0.9, 0), ("B", 0.8, 0), ("B", 0.95, 0), ("C", 0.7, 1),
                          ("C", 0.7, 1)])
    choice, how, runs = dy.switch_control(run, k=5)
    assert log == [("C", 50), ("B", 50), ("B", 100), ("C", 50), ("C", 100)]
    assert (choice, how) == ("C", "faster")


def test_switch_control_first_lock_in_the_initial_tests_decides():
    run, log = _scripted([("C", 0.6, 1), ("B", 0.5, 0)])
    assert dy.switch_control(run, k=5)[:2] == ("B", "faster")
    assert log == [("C", 50), ("B", 50)]


def test_switch_control_all_pairs_in_one_run():
    run, log = _scripted([("C", 0.1, 5)])
    assert dy.switch_control(run, k=5)[:2] == ("C", "found")
    run, log = _scripted([("C", 0.9, 0), ("B", 0.8, 0), ("B", 0.5, 5)])
    assert dy.switch_control(run, k=5)[:2] == ("B", "found")
    assert log == [("C", 50), ("B", 50), ("B", 100)]


def test_switch_control_switch_limit_and_halving():
    # B wins twice (j = 1, 2: 100, 200), then C (j = 1: 100), then B (j = 0: 50)
    run, log = _scripted([("C", 0.9, 0), ("B", 0.8, 0), ("B", 0.8, 0), ("B", 0.95, 0),
                          ("C", 0.99, 0), ("B", 0.9, 0)])
    choice, how, runs = dy.switch_control(run, k=3, max_switch=4)
    assert log == [("C", 50), ("B", 50), ("B", 100), ("B", 200), ("C", 100), ("B", 50)]
    assert (choice, how) == ("B", "faster") and len(runs) == 6


def test_segment_rate():
    logs = [0.0, math.log(0.5), math.log(0.25), None, 0.0, math.log(0.5)]
    assert dy.segment_rate(logs) == pytest.approx(0.5)
    assert dy.segment_rate([1.0]) == 1.0


def test_dynamic_on_the_switching_matrix():
    """diag([1:10, 1000:100:1e6]) with M = A + diag(rand * 1e4) (Section
    5.1), k = 1: sigma_1 = 1 exactly, to the residual test of Section 5."""
    A, mdiag = wl.switch_demo_matrix()
    Minv = lambda Y: Y / mdiag[:, None]
    out = dy.phsvds_dynamic(A, 1, 1e-12, precond=("inverse_A", Minv, Minv), anorm=1e6,
                            stage2_method="gdk")
    assert out["converged"]
    assert abs(out["sigma"][0] - 1.0) <= 1e-10
    assert dense.triplet_residuals(A, out["sigma"], out["U"], out["V"])[0] <= 1e-12 * 1e6
    assert out["dynamic"]["runs"][0][:2] == ("C", 50)


def _scrambled(sm_scale=None, seed=0, n=300):
    rng = np.random.default_rng(seed)
    Q1 = np.linalg.qr(rng.standard_normal((n, n)))[0]
    Q2 = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.concatenate([[1e-3, 2e-3, 3e-3], np.linspace(0.01, 1, n - 3)])
    sm = s.copy()
    for j, f in (sm_scale or {}).items():
        sm[j] *= f
    A = Q1 @ np.diag(s) @ Q2.T
    Mi = Q2 @ np.diag(1.0 / sm) @ Q1.T  # M = Q1 diag(sm) Q2^T
    return A, s, ("inverse_A", lambda Y: Mi @ Y, lambda X: Mi.T @ X)


@pytest.mark.parametrize("case,want", [("good", "C"), ("mismatch", "B")])
def test_dynamic_choice_follows_the_preconditioner(case, want):
    """M = A up to one singular value scaled by 1e-9 ('mismatch'): M^-1 M^-T
    amplifies that direction by 1e18 and C stalls while [0 M^-1; M^-T 0]
    still works on B; with M = A exactly ('good') C finishes in the first
    test.  Either way the three smallest triplets come out to 1e-12 ||A||."""
    A, s, pre = _scrambled({150: 1e-9} if case == "mismatch" else {})
    out = dy.phsvds_dynamic(A, 3, 1e-12, precond=pre, anorm=1.0, stage2_method="gdk")
    assert out["dynamic"]["choice"] == want
    assert out["converged"]
    assert np.allclose(out["sigma"], s[:3], rtol=1e-9, atol=0)
    assert np.all(dense.triplet_residuals(A, out["sigma"], out["U"], out["V"]) <= 1e-12)
