"""Seeded synthetic inputs for the PHSVDS hot path.

This module only builds inputs: sparse matrices, initial blocks and the
random draws the method consumes.  It holds none of the method's
arithmetic, so both the CPU oracle and the GPU path (through its tests and
benchmark) can take their inputs from here without sharing any solver code.

Every generator is deterministic in its seed (NumPy PCG64).  Matrices are
returned as ``scipy.sparse.csr_matrix`` in float64 with sorted,
duplicate-free column indices.

Workload families (the paper measures on University of Florida collection
matrices, which are not available here; these families stand in for them,
with sizes in the range of the paper's large-scale set, Section 5.5):

* ``givens_scrambled``   A = R [D; 0] Q with R, Q products of random Givens
  rotations, so the singular values are exactly D.
* ``grid_gradient``      the 2-D grid gradient [I (x) D1; D1 (x) I] with the
  forward-difference D1, optionally with a random positive weight per row.
* ``random_sparse``      fixed nnz per row at uniform random columns, N(0,1)
  values, plus a small positive diagonal shift.
* ``powerlaw_sparse``    power-law nnz per row (shifted Zipf), N(0,1) values,
  plus the same diagonal shift.
* ``diag_matrix``        the paper's diagonal test matrices (Section 5.1).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "givens_scrambled",
    "grid_gradient",
    "random_sparse",
    "powerlaw_sparse",
    "diag_matrix",
    "table1_matrix",
    "switch_demo_matrix",
    "initial_block",
    "uniform_block",
    "zipf_shift_for_mean",
    "gnn_init_weights",
]


def _csr(A) -> sp.csr_matrix:
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return A


def _rotations(dim: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """Product of ``count`` Givens rotations on random distinct index pairs
    with angles uniform in [0, 2*pi), as an explicit dense orthogonal matrix."""
    G = np.eye(dim)
    for _ in range(count):
        i, j = rng.choice(dim, size=2, replace=False)
        a = rng.uniform(0.0, 2.0 * math.pi)
        c, s = math.cos(a), math.sin(a)
        gi = G[i].copy()
        gj = G[j]
        G[i] = c * gi - s * gj
        G[j] = s * gi + c * gj
    return G


def givens_scrambled(m: int = 1200, n: int = 1000, sigma=None, rot_left: int | None = None,
                     rot_right: int | None = None, seed: int = 1):
    """A = R [diag(sigma); 0] Q.

    ``sigma`` defaults to 1000 values log-spaced in [1e-4, 1] (ascending).
    ``rot_left``/``rot_right`` default to 3n rotations each.  Returns
    ``(A, sigma, U_exact, V_exact)`` where column i of ``U_exact`` (m x n) and
    ``V_exact`` (n x n) are the exact singular vectors of sigma[i].
    """
    if sigma is None:
        sigma = np.logspace(-4.0, 0.0, n)
    sigma = np.asarray(sigma, dtype=np.float64)
    assert sigma.shape == (n,) and m >= n
    rot_left = 3 * n if rot_left is None else rot_left
    rot_right = 3 * n if rot_right is None else rot_right
    rng = np.random.default_rng(seed)
    Q = _rotations(n, rot_right, rng)
    R = _rotations(m, rot_left, rng)
    Ad = (R[:, :n] * sigma[None, :]) @ Q
    A = _csr(Ad)
    return A, sigma, R[:, :n].copy(), Q.T.copy()


def _forward_difference(N: int) -> sp.csr_matrix:
    """(N+1) x N forward difference: row i is x_i - x_{i-1} with zero ends."""
    rows = np.concatenate([np.arange(N), np.arange(1, N + 1)])
    cols = np.concatenate([np.arange(N), np.arange(N)])
    vals = np.concatenate([np.ones(N), -np.ones(N)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N + 1, N))


def grid_gradient(N: int, weights: str | None = None, seed: int = 3) -> sp.csr_matrix:
    """[I (x) D1; D1 (x) I] of size 2N(N+1) x N^2.

    ``weights='lognormal'`` multiplies every row by an i.i.d. lognormal(0, 1)
    weight (one weight per row, boundary rows included).
    """
    D1 = _forward_difference(N)
    I = sp.identity(N, format="csr")
    A = sp.vstack([sp.kron(I, D1), sp.kron(D1, I)], format="csr")
    if weights == "lognormal":
        rng = np.random.default_rng(seed)
        w = rng.lognormal(0.0, 1.0, size=A.shape[0])
        A = sp.diags(w) @ A
    elif weights is not None:
        raise ValueError(weights)
    return _csr(A)


def _diag_shift(A: sp.csr_matrix, n: int, rng: np.random.Generator, lo: float, hi: float):
    d = rng.uniform(lo, hi, size=n)
    S = sp.csr_matrix((d, (np.arange(n), np.arange(n))), shape=A.shape)
    return _csr(A + S)


def _rows_from_lengths(m: int, n: int, lengths: np.ndarray, rng: np.random.Generator):
    """Uniform random distinct columns per row (duplicates re-drawn)."""
    lengths = np.minimum(lengths.astype(np.int64), n)
    rows = np.repeat(np.arange(m, dtype=np.int64), lengths)
    cols = rng.integers(0, n, size=rows.size, dtype=np.int64)
    for _ in range(64):
        key = rows * n + cols
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        idx = order[dup]
        cols[idx] = rng.integers(0, n, size=idx.size, dtype=np.int64)
    vals = rng.standard_normal(rows.size)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, n))


def random_sparse(m: int = 300_000, n: int = 200_000, nnz_per_row: int = 12, seed: int = 1000,
                  shift=(0.01, 0.1)) -> sp.csr_matrix:
    """Fixed nnz per row at uniform random distinct columns, N(0,1) values,
    plus A[j, j] += d_j with d_j ~ U[shift] for j < n."""
    rng = np.random.default_rng(seed)
    A = _rows_from_lengths(m, n, np.full(m, nnz_per_row), rng)
    return _diag_shift(A, n, rng, *shift)


def _zipf_pmf(kmax: int, exponent: float, q: float) -> np.ndarray:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = (k + q) ** (-exponent)
    return p / p.sum()


def zipf_shift_for_mean(mean: float, kmax: int = 2000, exponent: float = 2.0) -> float:
    """q such that P(k) ~ (k+q)^-exponent on [1, kmax] has the given mean."""
    k = np.arange(1, kmax + 1, dtype=np.float64)
    lo, hi = -0.999, 1000.0
    for _ in range(200):
        q = 0.5 * (lo + hi)
        if float((k * _zipf_pmf(kmax, exponent, q)).sum()) < mean:
            lo = q
        else:
            hi = q
    return 0.5 * (lo + hi)


def powerlaw_sparse(m: int = 4_000_000, n: int = 3_000_000, mean: float = 10.0, kmax: int = 2000,
                    exponent: float = 2.0, seed: int = 5, shift=(0.01, 0.1)) -> sp.csr_matrix:
    """Row lengths from the shifted Zipf law P(k) ~ (k+q)^-exponent on
    [1, kmax] with q chosen to give the requested mean; uniform random
    distinct columns; N(0,1) values; plus the diagonal shift of
    ``random_sparse`` so that no column is empty."""
    rng = np.random.default_rng(seed)
    q = zipf_shift_for_mean(mean, kmax, exponent)
    pmf = _zipf_pmf(kmax, exponent, q)
    lengths = rng.choice(np.arange(1, kmax + 1), size=m, p=pmf)
    A = _rows_from_lengths(m, n, lengths, rng)
    return _diag_shift(A, n, rng, *shift)


def diag_matrix(values) -> sp.csr_matrix:
    v = np.asarray(values, dtype=np.float64)
    return _csr(sp.diags(v))


def table1_matrix() -> sp.csr_matrix:
    """diag([1e-14, 1e-12, 1e-8:1e-8:4e-8, 1e-3:1e-3:1]) of Section 5.1
    (n = 1006, ||A|| = 1)."""
    vals = np.concatenate([[1e-14, 1e-12], 1e-8 * np.arange(1, 5), 1e-3 * np.arange(1, 1001)])
    return diag_matrix(vals)


def switch_demo_matrix(seed: int = 7):
    """diag([1:10, 1000:100:1e6]) of Section 5.1 with its preconditioner
    diagonal A + rand*1e4 (the random draw is taken at the matrix size)."""
    vals = np.concatenate([np.arange(1, 11, dtype=np.float64), np.arange(1000.0, 1e6 + 1, 100.0)])
    rng = np.random.default_rng(seed)
    return diag_matrix(vals), vals + rng.random(vals.size) * 1e4


def initial_block(n: int, b: int, seed: int = 2) -> np.ndarray:
    """Initial block [ones/sqrt(n), randn(n, b-1)] (column-major, float64).

    The first column is the paper's ones(min(m, n), 1) start (Section 5);
    the other columns are seeded N(0, 1) draws."""
    X = np.empty((n, b), dtype=np.float64, order="F")
    X[:, 0] = 1.0 / math.sqrt(n)
    if b > 1:
        X[:, 1:] = np.random.default_rng(seed).standard_normal((n, b - 1))
    return X


def uniform_block(n: int, b: int, seed: int) -> np.ndarray:
    """Seeded U(-0.5, 0.5) block, used where the method needs random
    vectors (replacements for dependent columns, random left vectors)."""
    return np.asfortranarray(np.random.default_rng(seed).uniform(-0.5, 0.5, size=(n, b)))


def gnn_init_weights(width: int = 32, nin: int = 4, seed: int = 0) -> dict:
    """Initial weights of the message-passing preconditioner: Glorot-uniform
    matrices, zero biases, float32-representable values (the network trains
    in float32).  Layout and names: Ws1, Wm1 (nin x width), b1, then Ws2,
    Wm2, b2, Ws3, Wm3, b3 (width x width / width), then wo (width)."""
    rng = np.random.default_rng(seed)

    def glorot(fi, fo):
        lim = math.sqrt(6.0 / (fi + fo))
        return rng.uniform(-lim, lim, size=(fi, fo)).astype(np.float32).astype(np.float64)

    w = width
    P = {"Ws1": glorot(nin, w), "Wm1": glorot(nin, w), "b1": np.zeros(w)}
    for l in (2, 3):
        P[f"Ws{l}"] = glorot(w, w)
        P[f"Wm{l}"] = glorot(w, w)
        P[f"b{l}"] = np.zeros(w)
    P["wo"] = glorot(w, 1)[:, 0]
    return P


def inverse_poly_coeffs(hi: float, deg: int = 3, npts: int = 2000) -> np.ndarray:
    """Coefficients c_0..c_deg of the polynomial p minimising the sum of
    (x p(x) - 1)^2 over npts points spread evenly on (0, hi]: a polynomial
    approximation of 1/x on the spectrum of a positive operator whose largest
    eigenvalue is at most hi.  (With hi below the largest eigenvalue, p can
    turn negative there.)"""
    xs = np.linspace(hi / npts, hi, npts)
    V = np.vander(xs, deg + 1, increasing=True)
    return np.linalg.lstsq(V * xs[:, None], np.ones_like(xs), rcond=None)[0]


def gnn_poly_weights(coeffs, width: int = 32, nin: int = 4) -> dict:
    """Weights that make the message-passing preconditioner the polynomial
    p(Ch) = sum_k coeffs[k] Ch^k applied to its first input feature u (at
    most degree 3: one power of Ch per layer).  Channels 2k and 2k+1 of the
    layers carry relu(Ch^k u) and relu(-Ch^k u), so every layer stays linear
    in u; the readout takes coeffs[k] (relu(Ch^k u) - relu(-Ch^k u)) and
    coeffs[0] is lowered by one for the Jacobi feature the readout adds.
    Other channels, all biases and the d, tau inputs are zero."""
    c = [float(x) for x in coeffs]
    assert 1 <= len(c) <= 4 and width >= 2 * len(c)
    P = {"Ws1": np.zeros((nin, width)), "Wm1": np.zeros((nin, width)), "b1": np.zeros(width)}
    for l in (2, 3):
        P[f"Ws{l}"] = np.zeros((width, width))
        P[f"Wm{l}"] = np.zeros((width, width))
        P[f"b{l}"] = np.zeros(width)
    P["Ws1"][0, 0], P["Ws1"][0, 1] = 1.0, -1.0          # u, -u
    P["Wm1"][0, 2], P["Wm1"][0, 3] = 1.0, -1.0          # Ch u, -Ch u
    for l, top in ((2, 4), (3, 6)):
        for ch in range(top):                            # carry the lower powers
            P[f"Ws{l}"][ch, ch] = 1.0
        a = top - 2                                      # the highest power so far
        P[f"Wm{l}"][a, top], P[f"Wm{l}"][a + 1, top] = 1.0, -1.0
        P[f"Wm{l}"][a, top + 1], P[f"Wm{l}"][a + 1, top + 1] = -1.0, 1.0
    P["wo"] = np.zeros(width)
    c[0] -= 1.0
    for k, ck in enumerate(c):
        P["wo"][2 * k], P["wo"][2 * k + 1] = ck, -ck
    return P
