"""Tall-skinny products of the block iteration through the C ABI
(phsvds_tsgemm_tn / _nn): X^T Y on the matrix cores for long operands, the
vector kernels below 65536 rows, and X S, against NumPy in float64.

Inputs are drawn from U(0.5, 1.5), so every entry of the result is of the
size of |X|^T |Y| and a wrong operand layout shows as an O(1) relative
error; the bars are the forward-error bounds of the accumulation precision
(float32: partial sums over a block of rows in float32, blocks in float64)."""
import numpy as np
import pytest
import torch

from tests.gpu_util import as_np, gpu, need_gpu, say

TN_CASES = [
    # rows, nx, ny, y row-major
    (1000, 8, 8, True), (70000, 1, 1, False), (70000, 8, 8, True), (70000, 17, 3, False),
    (300001, 40, 8, True), (300001, 76, 8, True), (300001, 128, 16, False),
    (300001, 64, 16, True), (200003, 33, 24, False),
]


@gpu
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("rows,nx,ny,yrm", TN_CASES)
def test_tsgemm_tn_vs_numpy(rows, nx, ny, yrm, dtype):
    need_gpu()
    import paper_1408_5535_amd as P
    rng = np.random.default_rng(rows + nx + ny)
    X = rng.uniform(0.5, 1.5, (nx, rows))
    Y = rng.uniform(0.5, 1.5, (rows, ny) if yrm else (ny, rows))
    dt = torch.float32 if dtype == "float32" else torch.float64
    Xd = torch.tensor(X, dtype=dt, device="cuda")
    Yd = torch.tensor(Y, dtype=dt, device="cuda")
    say("tsgemm_tn", rows, nx, ny, "row-major Y" if yrm else "column-major Y", dtype)
    G = as_np(P.tsgemm_tn(Xd, Yd, y_row_major=yrm))
    Xr = Xd.double().cpu().numpy()
    Yr = Yd.double().cpu().numpy()
    ref = Xr @ (Yr if yrm else Yr.T)
    rel = np.max(np.abs(G - ref) / ref)
    say("  max relative error", rel)
    assert rel < (2e-4 if dtype == "float32" else 1e-12)


@gpu
@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_tsgemm_tn_signed_data_and_ragged_tail(dtype):
    """Signed N(0,1) data, a tail of rows below one LDS chunk: within the
    forward-error bound n eps |X|^T |Y| with n the rows."""
    need_gpu()
    import paper_1408_5535_amd as P
    rows, nx, ny = 65536 + 37, 50, 8
    rng = np.random.default_rng(5)
    X = rng.standard_normal((nx, rows))
    Y = rng.standard_normal((rows, ny))
    dt = torch.float32 if dtype == "float32" else torch.float64
    Xd = torch.tensor(X, dtype=dt, device="cuda")
    Yd = torch.tensor(Y, dtype=dt, device="cuda")
    G = as_np(P.tsgemm_tn(Xd, Yd, y_row_major=True))
    Xr, Yr = Xd.double().cpu().numpy(), Yd.double().cpu().numpy()
    eps = 2.0 ** -24 if dtype == "float32" else 2.0 ** -53
    bound = np.abs(Xr) @ np.abs(Yr) * rows * eps
    assert np.all(np.abs(G - Xr @ Yr) <= bound)


@gpu
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("beta", [-0.5, 0.0])
@pytest.mark.parametrize("rows,nx,ny,pad", [(70000, 8, 8, 0), (300001, 56, 42, 0),
                                             (300001, 50, 42, 7), (300001, 76, 8, 0),
                                             (65536 + 37, 64, 64, 0), (100003, 80, 20, 0),
                                             (99999, 5, 17, 0), (262144, 33, 25, 0),
                                             (100003, 33, 25, 3)])
def test_tsgemm_nn_vs_numpy(rows, nx, ny, pad, beta, dtype):
    """Y = alpha X S + beta Y against float64 numpy.  With pad > 0 the
    columns of X and Y sit in longer columns (leading dimension rows + pad):
    X's padding holds NaN, which no stored output may see, and Y's padding
    must come back untouched; beta = 0 is the plain product of the
    restarts."""
    need_gpu()
    import paper_1408_5535_amd as P
    rng = np.random.default_rng(rows + nx)
    X = rng.uniform(0.5, 1.5, (nx, rows))
    S = rng.uniform(0.5, 1.5, (nx, ny))
    Y0 = rng.uniform(0.5, 1.5, (ny, rows))
    dt = torch.float32 if dtype == "float32" else torch.float64
    Xf = torch.full((nx, rows + pad), float("nan"), dtype=dt, device="cuda")
    Yf = torch.full((ny, rows + pad), 7.0, dtype=dt, device="cuda")
    Xd, Yd = Xf[:, :rows], Yf[:, :rows]
    Xd.copy_(torch.tensor(X, dtype=dt))
    Yd.copy_(torch.tensor(Y0, dtype=dt))
    Sd = torch.tensor(S, dtype=torch.float64, device="cuda")
    Y0r = Yd.double().cpu().numpy()
    P.tsgemm_nn(Xd, Sd, Yd, alpha=0.75, beta=beta)
    ref = 0.75 * (S.T @ Xd.double().cpu().numpy()) + beta * Y0r
    got = Yd.double().cpu().numpy()
    scale = 0.75 * (S.T @ np.abs(Xd.double().cpu().numpy())) + abs(beta) * np.abs(Y0r)
    assert np.max(np.abs(got - ref) / scale) < (2e-6 * nx if dtype == "float32" else 1e-14 * nx)
    if pad:
        assert torch.all(Yf[:, rows:] == 7.0)


@gpu
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("rows,nx,ny", [(300001, 50, 42), (300002, 50, 42), (262144 + 5, 33, 25),
                                         (262144, 33, 25), (70001, 5, 17)])
def test_tsgemm_nn_reads_and_writes_only_its_columns(rows, nx, ny, dtype):
    """X and Y are the leading columns of wider tensors whose further
    columns hold NaN (X) or a sentinel (Y): the product's loads past
    column nx must read zero, not the neighbours, and its stores must stay
    within Y's ny columns (plain product and with beta)."""
    need_gpu()
    import paper_1408_5535_amd as P
    rng = np.random.default_rng(rows + 3 * nx)
    dt = torch.float32 if dtype == "float32" else torch.float64
    X = rng.uniform(0.5, 1.5, (nx, rows))
    S = rng.uniform(0.5, 1.5, (nx, ny))
    Xf = torch.full((nx + 3, rows), float("nan"), dtype=dt, device="cuda")
    Xf[:nx].copy_(torch.tensor(X, dtype=dt))
    Sd = torch.tensor(S, dtype=torch.float64, device="cuda")
    Xr = Xf[:nx].double().cpu().numpy()
    for beta in (0.0, 0.5):
        Yf = torch.full((ny + 2, rows), 7.0, dtype=dt, device="cuda")
        Yf[:ny].fill_(1.0)
        P.tsgemm_nn(Xf[:nx], Sd, Yf[:ny], alpha=1.0, beta=beta)
        got = Yf[:ny].double().cpu().numpy()
        ref = S.T @ Xr + beta
        scale = S.T @ np.abs(Xr) + beta
        assert np.all(np.isfinite(got))
        assert np.max(np.abs(got - ref) / scale) < (2e-6 * nx if dtype == "float32" else 1e-14 * nx)
        assert torch.all(Yf[ny:] == 7.0)


@gpu
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("rows,nb", [(300001, 8), (65536, 8), (100003, 6), (70001, 16), (5000, 8)])
def test_tsgemm_tn_row_major_gram(rows, nb, dtype):
    """G = X^T X of a row-major block (the CholQR Gram matrices of the
    solver): width 8 from 65536 rows takes the Gram kernel, the others the
    general products with a row-major X; against float64 numpy within the
    forward-error bound of the sums."""
    need_gpu()
    import paper_1408_5535_amd as P
    rng = np.random.default_rng(rows + nb)
    dt = torch.float32 if dtype == "float32" else torch.float64
    Xd = torch.tensor(rng.standard_normal((rows, nb)), dtype=dt, device="cuda")
    G = as_np(P.tsgemm_tn(Xd, Xd, y_row_major=True, x_row_major=True))
    Xr = Xd.double().cpu().numpy()
    eps = 2.0 ** -24 if dtype == "float32" else 2.0 ** -53
    bound = np.abs(Xr).T @ np.abs(Xr) * rows * eps
    assert np.all(np.abs(G - Xr.T @ Xr) <= bound)
    if nb == 8 and rows >= 65536:
        assert np.array_equal(G, G.T)  # one sum per pair, written to both
