"""The allocation-free transposed product (phsvds_spmm_noalloc) against the
workspace entry point it varies (phsvds_spmm), through the C ABI: the same
kernels, so the outputs agree bit for bit; two calls in a row, the second
on a smaller matrix (the scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as wl
from tests.gpu_util import gpu, need_gpu, say, to_dev


def _lib():
    import paper_1408_5535_amd as P
    lib = P._lib
    lib.phsvds_spmm_noalloc.argtypes = [ctypes.POINTER(P._Csr), ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
    return P, lib


def _both(P, lib, A, X, trans, fp32):
    D = to_dev(A)
    c = D._c()
    val32 = D.val.float() if fp32 else None
    rows_out = A.shape[1] if trans else A.shape[0]
    Y1 = torch.full((rows_out, X.shape[1]), float("nan"), dtype=X.dtype, device="cuda")
    Y2 = torch.full_like(Y1, float("nan"))
    nb = int(lib.phsvds_spmm_ws_bytes(ctypes.byref(c), int(trans), int(fp32)))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    s = P._stream()
    vp = val32.data_ptr() if val32 is not None else None
    rc = lib.phsvds_spmm(ctypes.byref(c), vp, int(trans), int(fp32), X.shape[1], X.data_ptr(),
                         Y1.data_ptr(), ws.data_ptr(), nb, s)
    assert rc == 0, lib.phsvds_last_error()
    rc = lib.phsvds_spmm_noalloc(ctypes.byref(c), vp, int(trans), int(fp32), X.shape[1],
                                 X.data_ptr(), Y2.data_ptr(), s)
    assert rc == 0, lib.phsvds_last_error()
    torch.cuda.synchronize()
    return Y1.cpu().numpy(), Y2.cpu().numpy()


@gpu
@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_matches_workspace_entry_two_calls(fp32):
    need_gpu()
    P, lib = _lib()
    dt = torch.float32 if fp32 else torch.float64
    cases = [("first, larger", wl.powerlaw_sparse(40000, 30000, kmax=500, seed=41), 8),
             ("second, smaller", wl.random_sparse(3000, 2000, 7, seed=42), 4)]
    for name, A, b in cases:
        for trans in (True, False):
            rows_in = A.shape[0] if trans else A.shape[1]
            X = torch.tensor(np.random.default_rng(43).standard_normal((rows_in, b)), dtype=dt,
                             device="cuda").contiguous()
            say("noalloc", name, "fp32", fp32, "trans", trans, "nnz", A.nnz)
            Y1, Y2 = _both(P, lib, A, X, trans, fp32)
            assert np.all(np.isfinite(Y1))
            assert np.array_equal(Y1, Y2)
            ref = (A.T if trans else A) @ X.cpu().double().numpy()
            bound = (abs(A.T if trans else A) @ np.abs(X.cpu().double().numpy())) * 600 * (
                2.0 ** -23 if fp32 else 2.0 ** -53)
            assert np.all(np.abs(Y2 - ref) <= bound + 1e-30)


@gpu
def test_noalloc_rejects_a_product_above_its_scratch():
    """A transposed product that needs more than the scratch is refused on
    the host (PHSVDS_ENOMEM) before any device access."""
    need_gpu()
    P, lib = _lib()
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    c = P._Csr(10_000_000, 8_000_000, 100_000_000, dummy.data_ptr(), dummy.data_ptr(),
               dummy.data_ptr())
    rc = lib.phsvds_spmm_noalloc(ctypes.byref(c), None, 1, 0, 1, dummy.data_ptr(),
                                 dummy.data_ptr(), P._stream())
    assert rc == -4
    assert b"scratch" in lib.phsvds_last_error()
