"""Closed-form spectra of the synthetic workloads (test infrastructure).

grid gradient [I (x) D1; D1 (x) I] with the (N+1) x N forward difference D1:
D1^T D1 = tridiag(-1, 2, -1) has eigenvalues 4 sin^2(i pi / (2(N+1))) with
eigenvectors s_i(p) = sqrt(2/(N+1)) sin(i p pi / (N+1)), so A^T A = I (x) T +
T (x) I has eigenvalues lambda_i + lambda_j and singular values
sigma_ij = sqrt(lambda_i + lambda_j).
"""
import numpy as np


def grid_lambdas(N):
    i = np.arange(1, N + 1)
    return 4.0 * np.sin(i * np.pi / (2.0 * (N + 1))) ** 2


def grid_sigmas(N):
    lam = grid_lambdas(N)
    return np.sort(np.sqrt((lam[:, None] + lam[None, :]).ravel()))


def grid_norm(N):
    lam = grid_lambdas(N)
    return float(np.sqrt(2.0 * lam[-1]))


def grid_sine(N, i):
    p = np.arange(1, N + 1)
    return np.sqrt(2.0 / (N + 1)) * np.sin(i * p * np.pi / (N + 1))


def principal_angles(X, Y):
    """Sine of the largest principal angle between span(X) and span(Y)
    (equal dimensions): ||(I - Qx Qx^T) Qy||_2, accurate for tiny angles."""
    Qx, _ = np.linalg.qr(X)
    Qy, _ = np.linalg.qr(Y)
    D = Qy - Qx @ (Qx.T @ Qy)
    return float(np.linalg.norm(D, 2))


def clusters(sig, rel=1e-8):
    """Group sorted values into clusters of relative spread < rel."""
    groups, cur = [], [0]
    for i in range(1, len(sig)):
        if abs(sig[i] - sig[cur[-1]]) <= rel * max(abs(sig[i]), 1e-300):
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    return groups
