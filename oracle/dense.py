"""Dense reference routines (float64).

* ``jacobi_svd``: one-sided Jacobi (Hestenes) SVD, the textbook routine.  It
  is the plain definition of the singular triplets of Section 1, eq. (1),
  on inputs small enough to densify.  Pinned against LAPACK
  (numpy.linalg.svd) and against closed-form spectra in the tests.
* ``svd_extreme_dense``: the k smallest (or largest) triplets via
  ``jacobi_svd``, sorted, with the sign convention of the library output.
* ``triplet_residuals``: the stopping quantity of Section 5,
  sqrt(||r_u||^2 + ||r_v||^2) with r_v = A v - sigma u, r_u = A^T u - sigma v
  (eq. "different residuals", Section 3.1).
"""
from __future__ import annotations

import numpy as np


def jacobi_svd(A: np.ndarray, tol: float = 2.0 ** -52, max_sweeps: int = 60):
    """One-sided Jacobi SVD of a dense m x n matrix (m >= n).

    Rotates pairs of columns of G = A V until every pair is orthogonal to
    working precision; then sigma_j = ||G_:,j||, u_j = G_:,j / sigma_j and V
    accumulates the rotations.  Returns (U, s, V) with s descending, the
    same convention as LAPACK's gesvd.  Columns with s_j == 0 get u_j = 0.
    """
    G = np.array(A, dtype=np.float64, copy=True)
    m, n = G.shape
    if m < n:
        raise ValueError("jacobi_svd expects m >= n")
    V = np.eye(n)
    for _ in range(max_sweeps):
        rotated = False
        for i in range(n - 1):
            for j in range(i + 1, n):
                gi, gj = G[:, i], G[:, j]
                alpha = gi @ gi
                beta = gj @ gj
                gamma = gi @ gj
                if gamma == 0.0 or abs(gamma) <= tol * np.sqrt(alpha * beta):
                    continue
                rotated = True
                zeta = (beta - alpha) / (2.0 * gamma)
                t = np.sign(zeta) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta)) if zeta != 0 else 1.0
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = c * t
                Gi = gi.copy()
                G[:, i] = c * Gi - s * gj
                G[:, j] = s * Gi + c * gj
                Vi = V[:, i].copy()
                V[:, i] = c * Vi - s * V[:, j]
                V[:, j] = s * Vi + c * V[:, j]
        if not rotated:
            break
    s = np.sqrt(np.einsum("ij,ij->j", G, G))
    order = np.argsort(-s, kind="stable")
    s = s[order]
    G = G[:, order]
    V = V[:, order]
    U = np.zeros_like(G)
    nz = s > 0
    U[:, nz] = G[:, nz] / s[nz]
    return U, s, V


def _sign_normalise(U: np.ndarray, V: np.ndarray):
    """Make the largest-magnitude entry of each v_i positive (u_i follows)."""
    for i in range(V.shape[1]):
        j = np.argmax(np.abs(V[:, i]))
        if V[j, i] < 0:
            V[:, i] *= -1.0
            U[:, i] *= -1.0
    return U, V


def svd_extreme_dense(A, k: int, which: str = "smallest"):
    """The k smallest (ascending) or largest (descending) singular triplets
    of A by the dense one-sided Jacobi SVD.  Returns (sigma, U, V)."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A, dtype=np.float64)
    U, s, V = jacobi_svd(Ad)
    if which == "smallest":
        idx = np.arange(len(s) - 1, len(s) - 1 - k, -1)
    elif which == "largest":
        idx = np.arange(k)
    else:
        raise ValueError(which)
    sig = s[idx].copy()
    Uk = U[:, idx].copy()
    Vk = V[:, idx].copy()
    Uk, Vk = _sign_normalise(Uk, Vk)
    return sig, Uk, Vk


def triplet_residuals(A, sigma, U, V) -> np.ndarray:
    """sqrt(||A v - sigma u||^2 + ||A^T u - sigma v||^2) per triplet, float64."""
    sigma = np.asarray(sigma, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    rv = A @ V - U * sigma[None, :]
    ru = A.T @ U - V * sigma[None, :]
    return np.sqrt((rv * rv).sum(0) + (ru * ru).sum(0))
