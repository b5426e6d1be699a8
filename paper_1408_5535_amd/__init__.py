"""MI355X PHSVDS: Python binding of libphsvds.so (argument marshalling only).

Every numerical step runs in the library's HIP kernels; PyTorch supplies
device memory and the current HIP stream.  There is no CPU fallback: if the
library is not built, importing this package raises.

The names follow the C ABI in include/phsvds.h:
    svds_smallest(A, k, tol, precond) -> (sigma, U, V, info)   (phsvds_svds)
    spmm(A, X)                        -> A X                   (phsvds_spmm_*)
    csr_transpose(A)                  -> A^T                   (phsvds_csr_transpose)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # noqa: F401  (loads the HIP runtime the library shares)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphsvds.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run python paper_1408_5535_amd/build.py first")
_lib = ctypes.CDLL(LIB_PATH)

PHSVDS_OK = 0
PHSVDS_NOT_CONVERGED = 1
PREC = {"none": 0, "jacobi": 1, "gnn": 2, "user": 3, "user_A": 4}
PHSVDS_EUSER = -5

# int (*)(void *ctx, const void *R, void *T, int64_t n, int b, const double *theta,
#         int fp64, void *stream)
USER_APPLY = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                              ctypes.c_int, ctypes.c_void_p)


# int (*)(void *ctx, const void *X, void *Y, int b, int trans, int fp64, void *stream)
USER_SOLVE = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p)


class _Csr(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class _Precond(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("gnn_weights", ctypes.c_void_p),
                ("gnn_width", ctypes.c_int), ("fallback_window", ctypes.c_int),
                ("user_apply", USER_APPLY), ("user_ctx", ctypes.c_void_p),
                ("user_solve", USER_SOLVE), ("user_apply_B", USER_APPLY)]


# int (*)(void *ctx, const void *X, void *Y, int b, int fp64, void *stream)
C_APPLY = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_int, ctypes.c_int, ctypes.c_void_p)


class _Opts(ctypes.Structure):
    _fields_ = [("which", ctypes.c_int), ("block", ctypes.c_int), ("max_basis", ctypes.c_int),
                ("min_restart", ctypes.c_int), ("stage1_fp32", ctypes.c_int),
                ("fp64_continue", ctypes.c_int), ("stage2", ctypes.c_int),
                ("max_restarts", ctypes.c_int), ("max_matvecs", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("init_block", ctypes.c_void_p),
                ("anorm", ctypes.c_double), ("floor_factor", ctypes.c_double),
                ("gnn_width", ctypes.c_int), ("verbose", ctypes.c_int),
                ("stage2_method", ctypes.c_int), ("max_inner", ctypes.c_int),
                ("init_V", ctypes.c_void_p), ("k0", ctypes.c_int),
                ("shifts", ctypes.POINTER(ctypes.c_double)), ("dynamic", ctypes.c_int),
                ("init_iter", ctypes.c_int), ("max_switch", ctypes.c_int),
                ("c_apply", C_APPLY), ("c_ctx", ctypes.c_void_p), ("c_inverse", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ("mv_stage1", "mv_rr", "mv_stage2", "mv_final", "mv_prec", "mv_floor",
                 "iters1", "iters2", "restarts1", "restarts2", "stage2_pairs", "fp32_locked",
                 "fallbacks", "refreshes", "rollbacks", "inner2")] + \
               [(f, ctypes.c_double) for f in
                ("t_setup", "t_stage1", "t_stage2", "t_total", "anorm_est")] + \
               [("res_stage1", ctypes.c_double * 64)] + \
               [(f, ctypes.c_int64) for f in ("dyn_choice", "dyn_found", "dyn_runs")] + \
               [(f, ctypes.c_int64 * 16) for f in ("dyn_on", "dyn_iters", "dyn_locked")] + \
               [("dyn_rate", ctypes.c_double * 16)] + \
               [("dep_cols", ctypes.c_int64)]

    _ARRAYS = ("res_stage1", "dyn_on", "dyn_iters", "dyn_locked", "dyn_rate")

    def as_dict(self, k):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in self._ARRAYS}
        d["res_stage1"] = list(self.res_stage1[:k])
        d["mv_total"] = self.mv_stage1 + self.mv_rr + self.mv_stage2 + self.mv_final
        if self.dyn_choice:
            nr = min(self.dyn_runs, 16)
            d["dynamic"] = {
                "choice": "CB"[self.dyn_choice - 1], "how": "found" if self.dyn_found else "faster",
                "runs": [("CB"[self.dyn_on[i] - 1], self.dyn_iters[i], self.dyn_rate[i],
                          self.dyn_locked[i]) for i in range(nr)]}
        return d


_P = ctypes.c_void_p
_lib.phsvds_version.restype = ctypes.c_char_p
_lib.phsvds_last_error.restype = ctypes.c_char_p
_lib.phsvds_default_opts.argtypes = [ctypes.POINTER(_Opts)]
_lib.phsvds_spmm_f64.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, _P, _P, ctypes.c_int, _P]
_lib.phsvds_spmm_f32.argtypes = [ctypes.POINTER(_Csr), _P, ctypes.c_int, _P, _P, ctypes.c_int, _P]
_lib.phsvds_rr_eig.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P,
                               _P, ctypes.c_int, _P]
_lib.phsvds_small_svd.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P,
                                  ctypes.c_int, _P]
_lib.phsvds_transpose_ws_bytes.argtypes = [ctypes.POINTER(_Csr)]
_lib.phsvds_transpose_ws_bytes.restype = ctypes.c_size_t
_lib.phsvds_csr_transpose.argtypes = [ctypes.POINTER(_Csr), _P, _P, _P, _P, ctypes.c_size_t, _P]
_lib.phsvds_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int, ctypes.POINTER(_Opts),
                                        ctypes.POINTER(ctypes.c_size_t)]
_lib.phsvds_svds.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, ctypes.c_double,
                             ctypes.POINTER(_Precond), ctypes.POINTER(_Opts), _P, ctypes.c_size_t,
                             _P, _P, _P, _P, _P, ctypes.POINTER(_Stats)]
# int (*)(void *ctx, const void *X, void *Y, int b, int trans, int fp64, void *stream)
OP_APPLY = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p)


class _Operator(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("apply", OP_APPLY),
                ("ctx", ctypes.c_void_p)]


_lib.phsvds_svds_op.argtypes = [ctypes.POINTER(_Operator), ctypes.c_int, ctypes.c_double,
                                ctypes.POINTER(_Precond), ctypes.POINTER(_Opts), _P,
                                ctypes.c_size_t, _P, _P, _P, _P, _P, ctypes.POINTER(_Stats)]


_lib.phsvds_profile.argtypes = [ctypes.c_int]
_lib.phsvds_profile_sample.argtypes = [ctypes.c_int]
_lib.phsvds_profile_read.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
PROFILE_KINDS = {"spmm_f64": 0, "spmm_f32": 1, "tn": 2, "nn": 3, "ritz": 4}


def profile(enable: bool, kinds=None, every: int = 1) -> None:
    """Start (clearing counters) or stop event timing of the library's
    kernels; ``kinds`` (names or numbers) restricts the timed kinds, and
    ``every`` > 1 times one pair of consecutive operations in ``every``."""
    code = int(bool(enable))
    if enable and kinds is not None:
        code = sum(1 << ((PROFILE_KINDS[k] if isinstance(k, str) else k) + 1) for k in kinds)
    _check(_lib.phsvds_profile(code), "profile")
    if enable:
        _check(_lib.phsvds_profile_sample(int(every)), "profile")


def profile_read(kind) -> tuple:
    """(timed operations, device seconds, algorithmic bytes) for a kind."""
    if isinstance(kind, str):
        kind = PROFILE_KINDS[kind]
    n = ctypes.c_int64(0)
    s = ctypes.c_double(0)
    b = ctypes.c_double(0)
    _check(_lib.phsvds_profile_read(kind, ctypes.byref(n), ctypes.byref(s), ctypes.byref(b)),
           "profile_read")
    return int(n.value), float(s.value), float(b.value)


def version() -> str:
    return _lib.phsvds_version().decode()


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"{what} failed ({rc}): {_lib.phsvds_last_error().decode()}")
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Operator:
    """A given by its products (Section 3.3): ``apply(X, Y, trans)`` fills
    Y = A X (trans False; X n x b, Y m x b) or A^T X (trans True; X m x b,
    Y n x b), torch float64 views of the library's row-major blocks."""

    nnz = 0

    def __init__(self, m, n, apply):
        self.m, self.n, self.apply = int(m), int(n), apply
        self.rowptr = torch.empty(0, device="cuda")  # device of the workspace

    def _c(self):
        m, n, fn = self.m, self.n, self.apply

        def call(ctx, X, Y, b, trans, fp64, stream):
            try:
                rin, rout = (m, n) if trans else (n, m)
                Xt = torch.as_tensor(_DevView(X, (rin, b), "f8"), device="cuda")
                Yt = torch.as_tensor(_DevView(Y, (rout, b), "f8"), device="cuda")
                fn(Xt, Yt, bool(trans))
                return 0
            except Exception:  # reported to the library as a nonzero return
                return 1
        self._cb = OP_APPLY(call)
        return _Operator(m, n, self._cb, None)


@dataclass
class DeviceCSR:
    """CSR matrix on the GPU: rowptr int64 (m+1), colind int32, val float64."""
    m: int
    n: int
    rowptr: torch.Tensor
    colind: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self):
        return int(self.colind.numel())

    @classmethod
    def from_scipy(cls, A, device="cuda"):
        A = A.tocsr()
        A.sort_indices()
        return cls(A.shape[0], A.shape[1],
                   torch.as_tensor(A.indptr.astype("int64")).to(device),
                   torch.as_tensor(A.indices.astype("int32")).to(device),
                   torch.as_tensor(A.data.astype("float64")).to(device))

    def _c(self):
        assert self.rowptr.dtype == torch.int64 and self.colind.dtype == torch.int32
        assert self.val.dtype == torch.float64 and self.rowptr.is_cuda
        return _Csr(self.m, self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr(),
                    self.val.data_ptr())


def spmm(A: DeviceCSR, X: torch.Tensor, absval: bool = False, val32: torch.Tensor | None = None):
    """Y = A X for a row-major block X (n x b, b in 1,2,4,8,16,32), float64
    or float32 (then ``val32`` holds the float32 values of A)."""
    assert X.is_cuda and X.is_contiguous() and X.shape[0] == A.n
    b = 1 if X.dim() == 1 else X.shape[1]
    Y = torch.empty((A.m,) + tuple(X.shape[1:]), dtype=X.dtype, device=X.device)
    c = A._c()
    if X.dtype == torch.float64:
        _check(_lib.phsvds_spmm_f64(ctypes.byref(c), b, X.data_ptr(), Y.data_ptr(), int(absval),
                                    _stream()), "spmm")
    elif X.dtype == torch.float32:
        if val32 is None:
            val32 = A.val.float()
        _check(_lib.phsvds_spmm_f32(ctypes.byref(c), val32.data_ptr(), b, X.data_ptr(),
                                    Y.data_ptr(), int(absval), _stream()), "spmm")
    else:
        raise TypeError(X.dtype)
    return Y


_lib.phsvds_spmm_ws_bytes.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, ctypes.c_int]
_lib.phsvds_spmm_ws_bytes.restype = ctypes.c_size_t
_lib.phsvds_spmm.argtypes = [ctypes.POINTER(_Csr), _P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             _P, _P, _P, ctypes.c_size_t, _P]


def spmm_op(A: DeviceCSR, X: torch.Tensor, trans: bool = False,
            val32: torch.Tensor | None = None):
    """Y = A X or A^T X (phsvds_spmm) for a row-major block X, float64 or
    float32 (val32: the float32 values of A for an untransposed product)."""
    assert X.is_cuda and X.is_contiguous()
    rows_in, rows_out = (A.m, A.n) if trans else (A.n, A.m)
    assert X.shape[0] == rows_in
    b = 1 if X.dim() == 1 else X.shape[1]
    fp32 = X.dtype == torch.float32
    Y = torch.empty((rows_out,) + tuple(X.shape[1:]), dtype=X.dtype, device=X.device)
    c = A._c()
    nb = int(_lib.phsvds_spmm_ws_bytes(ctypes.byref(c), int(trans), int(fp32)))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=X.device)
    if fp32 and not trans and val32 is None:
        val32 = A.val.float()
    _check(_lib.phsvds_spmm(ctypes.byref(c), val32.data_ptr() if val32 is not None else None,
                            int(trans), int(fp32), b, X.data_ptr(), Y.data_ptr(),
                            ws.data_ptr(), nb, _stream()), "spmm")
    return Y


_lib.phsvds_tsgemm_ws_bytes.restype = ctypes.c_size_t
_lib.phsvds_tsgemm_tn.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _P,
                                  ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int, _P,
                                  ctypes.c_int, _P, ctypes.c_size_t, _P]
_lib.phsvds_tsgemm_nn.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, _P, ctypes.c_int64, _P, ctypes.c_int,
                                  ctypes.c_double, _P, ctypes.c_int64, _P]


def tsgemm_tn(X: torch.Tensor, Y: torch.Tensor, y_row_major: bool = False,
              x_row_major: bool = False) -> torch.Tensor:
    """G = X^T Y (float64, nx x ny) for X (nx x rows storage: X[i] is column
    i, i.e. a column-major rows x nx matrix, or with x_row_major a rows x nx
    row-major tensor) and Y given the same way (or, with y_row_major, as a
    rows x ny row-major tensor)."""
    fp32 = X.dtype == torch.float32
    if x_row_major:
        rows, nx = X.shape
    else:
        nx, rows = X.shape
    if y_row_major:
        ny, ldy, layout = Y.shape[1], Y.stride(0), 0
    else:
        ny, ldy, layout = Y.shape[0], Y.stride(0), 1
    if x_row_major:
        layout |= 2
    G = torch.empty((ny, nx), dtype=torch.float64, device=X.device)  # column-major nx x ny
    ws = torch.empty(int(_lib.phsvds_tsgemm_ws_bytes()), dtype=torch.uint8, device=X.device)
    _check(_lib.phsvds_tsgemm_tn(int(fp32), rows, nx, ny, X.data_ptr(), X.stride(0),
                                 Y.data_ptr(), ldy, layout, G.data_ptr(), nx, ws.data_ptr(),
                                 ws.numel(), _stream()), "tsgemm_tn")
    return G.t()


def tsgemm_nn(X: torch.Tensor, S: torch.Tensor, Y: torch.Tensor, alpha=1.0, beta=0.0):
    """Y = alpha X S + beta Y in place, X (nx x rows storage, column-major),
    S (nx x ny float64), Y (ny x rows storage, column-major)."""
    fp32 = X.dtype == torch.float32
    nx, rows = X.shape
    ny = Y.shape[0]
    Sc = S.to(dtype=torch.float64).t().contiguous()  # column-major nx x ny
    _check(_lib.phsvds_tsgemm_nn(int(fp32), rows, nx, ny, float(alpha), X.data_ptr(),
                                 X.stride(0), Sc.data_ptr(), nx, float(beta), Y.data_ptr(),
                                 Y.stride(0), _stream()), "tsgemm_nn")
    return Y


_lib.phsvds_jacobi_ws_bytes.argtypes = [ctypes.POINTER(_Csr)]
_lib.phsvds_jacobi_ws_bytes.restype = ctypes.c_size_t
_lib.phsvds_jacobi_scaled_values.argtypes = [ctypes.POINTER(_Csr), _P, _P, ctypes.c_size_t, _P]


def jacobi_scaled(A: DeviceCSR) -> DeviceCSR:
    """A D^-1/2 with D = diag(A^T A), formed on the device (the operator
    whose squared largest singular value bounds the spectrum of the learned
    preconditioner's Ch)."""
    c = A._c()
    nb = int(_lib.phsvds_jacobi_ws_bytes(ctypes.byref(c)))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=A.val.device)
    out = torch.empty_like(A.val)
    _check(_lib.phsvds_jacobi_scaled_values(ctypes.byref(c), out.data_ptr(), ws.data_ptr(), nb,
                                            _stream()), "jacobi_scaled_values")
    return DeviceCSR(A.m, A.n, A.rowptr, A.colind, out)


def rr_eig(H: torch.Tensor, nvec: int, largest: bool = False):
    """Selected eigenpairs of the symmetric p x p device float64 matrix H
    (p <= 64): (theta (p,), S (p x p)); theta[:nvec], S[:, :nvec] are the
    nvec wanted pairs, theta[p-1] the eigenvalue at the other end, the rest
    NaN."""
    p = H.shape[0]
    Hc = H.to(dtype=torch.float64).t().contiguous()  # column-major
    theta = torch.full((p,), float("nan"), dtype=torch.float64, device=H.device)
    S = torch.full((p, p), float("nan"), dtype=torch.float64, device=H.device)
    _check(_lib.phsvds_rr_eig(Hc.data_ptr(), p, p, nvec, int(largest), theta.data_ptr(),
                              S.data_ptr(), p, _stream()), "rr_eig")
    return theta, S.t()


def small_svd(M: torch.Tensor):
    """Singular values (ascending, (cols,)) and right singular vectors
    (cols x cols, column j for sv[j]) of the small device float64 matrix M
    (rows x cols, cols <= 64, cols <= rows <= 128)."""
    rows, cols = M.shape
    Mc = M.to(dtype=torch.float64).t().contiguous()  # column-major
    sv = torch.empty(cols, dtype=torch.float64, device=M.device)
    Y = torch.empty((cols, cols), dtype=torch.float64, device=M.device)
    _check(_lib.phsvds_small_svd(Mc.data_ptr(), rows, rows, cols, sv.data_ptr(), Y.data_ptr(),
                                 cols, _stream()), "small_svd")
    return sv, Y.t()


def csr_transpose(A: DeviceCSR) -> DeviceCSR:
    c = A._c()
    dev = A.rowptr.device
    trp = torch.empty(A.n + 1, dtype=torch.int64, device=dev)
    tci = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    tva = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=dev)
    wsb = _lib.phsvds_transpose_ws_bytes(ctypes.byref(c))
    ws = torch.empty(max(int(wsb), 1), dtype=torch.uint8, device=dev)
    _check(_lib.phsvds_csr_transpose(ctypes.byref(c), trp.data_ptr(), tci.data_ptr(),
                                     tva.data_ptr(), ws.data_ptr(), wsb, _stream()), "transpose")
    return DeviceCSR(A.n, A.m, trp, tci[:A.nnz], tva[:A.nnz])


def make_opts(which="smallest", block=1, max_basis=0, min_restart=0, stage1_fp32=False,
              fp64_continue=True, stage2="auto", max_restarts=10000, max_matvecs=0, seed=1,
              init_block=None, anorm=0.0, floor_factor=10.0, gnn_width=0, verbose=False,
              stage2_method="jdqmr", max_inner=50, init_V=None, shifts=None, dynamic=False,
              init_iter=0, max_switch=0, c_apply=None, c_inverse=False, n=None):
    """Options of phsvds_svds.  ``c_apply(X, Y)`` (with ``n``, the columns
    of A) fills Y = C X, or C^-1 X with ``c_inverse`` (shift-invert), X and
    Y torch float64 views n x b of the library's row-major blocks."""
    o = _Opts()
    _lib.phsvds_default_opts(ctypes.byref(o))
    o.which = {"smallest": 0, "largest": 1}[which]
    o.block = block
    o.max_basis = max_basis
    o.min_restart = min_restart
    o.stage1_fp32 = int(stage1_fp32)
    o.fp64_continue = int(fp64_continue)
    o.stage2 = {"auto": 0, "force": 1, "never": -1}[stage2]
    o.max_restarts = max_restarts
    o.max_matvecs = max_matvecs
    o.seed = seed
    keep = None
    if init_block is not None:
        # (n x b) tensor -> n x b column-major device array
        keep = init_block.to(dtype=torch.float64, device="cuda").t().contiguous()
        o.init_block = keep.data_ptr()
    o.anorm = float(anorm)
    o.floor_factor = floor_factor
    o.gnn_width = gnn_width
    o.verbose = int(verbose)
    o.stage2_method = {"gdk": 0, "jdqmr": 1}[stage2_method]
    o.max_inner = max_inner
    o.dynamic = int(dynamic)
    o.init_iter = init_iter
    o.max_switch = max_switch
    keep4 = None
    if c_apply is not None:
        def call(ctx, X, Y, b, fp64, stream):
            try:
                Xt = torch.as_tensor(_DevView(X, (n, b), "f8"), device="cuda")
                Yt = torch.as_tensor(_DevView(Y, (n, b), "f8"), device="cuda")
                c_apply(Xt, Yt)
                return 0
            except Exception:  # reported to the library as a nonzero return
                return 1
        keep4 = C_APPLY(call)
        o.c_apply = keep4
        o.c_inverse = int(c_inverse)
    keep2 = None
    if init_V is not None:
        # (n x k0) tensor -> n x k0 column-major device array
        keep2 = init_V.to(dtype=torch.float64, device="cuda").t().contiguous()
        o.init_V = keep2.data_ptr()
        o.k0 = int(init_V.shape[1])
    keep3 = None
    if shifts is not None:
        keep3 = (ctypes.c_double * len(shifts))(*[float(x) for x in shifts])
        o.shifts = ctypes.cast(keep3, ctypes.POINTER(ctypes.c_double))
    o._keep = (keep, keep2, keep3, keep4)
    return o


def workspace_bytes(m, n, nnz, k, opts) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.phsvds_workspace_bytes(m, n, nnz, k, ctypes.byref(opts), ctypes.byref(out)),
           "workspace_bytes")
    return int(out.value)


class Solver:
    """Holds the workspace for repeated solves of one problem shape."""

    def __init__(self, A: DeviceCSR, k: int, **opt_kw):
        self.A, self.k = A, k
        if opt_kw.get("c_apply") is not None:
            opt_kw["n"] = A.n
        self.opts = make_opts(**opt_kw)
        nbytes = workspace_bytes(A.m, A.n, A.nnz, k, self.opts)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=A.rowptr.device)
        self.U = torch.empty((k, A.m), dtype=torch.float64, device=A.rowptr.device)
        self.V = torch.empty((k, A.n), dtype=torch.float64, device=A.rowptr.device)

    def solve(self, tol=1e-12, precond="none", gnn_weights=None, gnn_width=32,
              fallback_window=0, user_apply=None, user_solve=None, user_apply_B=None):
        """``user_apply(R, T, theta, fp64)`` (precond='user'): fills T = M R,
        R and T torch views (b x n, the rows are the columns of the C ABI's
        n x b column-major blocks), theta a list of b floats; a raised
        exception makes the call return nonzero.  ``user_apply_B(R, T,
        theta, fp64)`` (precond='user'): the same for a preconditioner of B
        itself, views b x (m + n).  ``user_solve(X, Y, trans, fp64)``
        (precond='user_A'): Y = M^-1 X (trans False; X b x m, Y b x n) or
        M^-T X (trans True; X b x n, Y b x m) for M ~ A."""
        import numpy as np
        k = self.k
        sig = (ctypes.c_double * k)()
        res = (ctypes.c_double * k)()
        st = _Stats()
        cb, cbs, cbB = USER_APPLY(), USER_SOLVE(), USER_APPLY()
        if precond == "user" and user_apply is not None:
            cb = USER_APPLY(_user_trampoline(user_apply))
        if precond == "user" and user_apply_B is not None:
            cbB = USER_APPLY(_user_trampoline(user_apply_B))
        if precond == "user_A":
            cbs = USER_SOLVE(_solve_trampoline(user_solve, self.A.m, self.A.n))
        pc = _Precond(PREC[precond], gnn_weights.data_ptr() if gnn_weights is not None else None,
                      gnn_width, fallback_window, cb, None, cbs, cbB)
        c = self.A._c()
        entry = _lib.phsvds_svds_op if isinstance(self.A, Operator) else _lib.phsvds_svds
        rc = entry(ctypes.byref(c), k, tol, ctypes.byref(pc), ctypes.byref(self.opts),
                   self.ws.data_ptr(), self.ws.numel(), _stream(), sig,
                   self.U.data_ptr(), self.V.data_ptr(), res, ctypes.byref(st))
        _check(rc, "svds")
        info = st.as_dict(k)
        info["status"] = rc
        info["res"] = np.array(res[:])
        # column-major m x k == row-major k x m: transpose views
        return np.array(sig[:]), self.U.T, self.V.T, info


class _DevView:
    """A device array handed over by pointer (no copy), for torch.as_tensor."""

    def __init__(self, ptr, shape, dtype):
        self.__cuda_array_interface__ = {"data": (int(ptr), False), "shape": tuple(shape),
                                         "typestr": "<f8" if dtype == "f8" else "<f4",
                                         "strides": None, "version": 2}


def _user_trampoline(fn):
    def call(ctx, R, T, n, b, theta, fp64, stream):
        try:
            dt = "f8" if fp64 else "f4"
            Rt = torch.as_tensor(_DevView(R, (b, n), dt), device="cuda")
            Tt = torch.as_tensor(_DevView(T, (b, n), dt), device="cuda")
            fn(Rt, Tt, [theta[i] for i in range(b)], bool(fp64))
            return 0
        except Exception:  # reported to the library as a nonzero return
            return 1
    return call


def _solve_trampoline(fn, m, n):
    def call(ctx, X, Y, b, trans, fp64, stream):
        try:
            dt = "f8" if fp64 else "f4"
            rin, rout = (n, m) if trans else (m, n)
            Xt = torch.as_tensor(_DevView(X, (b, rin), dt), device="cuda")
            Yt = torch.as_tensor(_DevView(Y, (b, rout), dt), device="cuda")
            fn(Xt, Yt, bool(trans), bool(fp64))
            return 0
        except Exception:  # reported to the library as a nonzero return
            return 1
    return call


def svds_smallest(A: DeviceCSR, k: int, tol: float = 1e-12, precond: str = "none",
                  gnn_weights=None, gnn_width=32, user_apply=None, user_solve=None,
                  user_apply_B=None, **opt_kw):
    """The k smallest (``which='largest'``: largest) singular triplets of A
    to sqrt(||r_u||^2 + ||r_v||^2) <= tol ||A||.  Returns
    (sigma, U (m x k), V (n x k), info)."""
    if precond == "gnn":
        opt_kw["gnn_width"] = gnn_width
    return Solver(A, k, **opt_kw).solve(tol, precond, gnn_weights, gnn_width,
                                        user_apply=user_apply, user_solve=user_solve,
                                        user_apply_B=user_apply_B)


# ---------------------------------------------------------------- learned preconditioner
GNN_NAMES = ["Ws1", "Wm1", "b1", "Ws2", "Wm2", "b2", "Ws3", "Wm3", "b3", "wo"]
_lib.phsvds_gnn_nweights.argtypes = [ctypes.c_int]
_lib.phsvds_gnn_nweights.restype = ctypes.c_int64
_lib.phsvds_gnn_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int]
_lib.phsvds_gnn_workspace_bytes.restype = ctypes.c_size_t
_lib.phsvds_gnn_prepare.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, _P, ctypes.c_size_t, _P]
_lib.phsvds_gnn_forward.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, _P, ctypes.c_size_t, _P,
                                    _P, _P, ctypes.c_double, _P, _P]
_lib.phsvds_gnn_loss_grad.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, _P, ctypes.c_size_t,
                                      _P, _P, _P, ctypes.c_double, _P, _P, _P, _P]
_lib.phsvds_gnn_residual_loss_grad.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, _P,
                                               ctypes.c_size_t, _P, _P, _P, ctypes.c_double, _P,
                                               _P, _P]
_lib.phsvds_gnn_adam.argtypes = [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, _P]
_lib.phsvds_harvest_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_int, ctypes.POINTER(_Opts),
                                                ctypes.POINTER(ctypes.c_size_t)]
_lib.phsvds_harvest.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                ctypes.POINTER(_Opts), _P, ctypes.c_size_t, _P, _P, _P, _P,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(_Stats)]


def gnn_nweights(width: int = 32) -> int:
    return int(_lib.phsvds_gnn_nweights(width))


def gnn_pack(params: dict, device="cuda") -> torch.Tensor:
    """Weights dict (row-major fin x w matrices) -> flat float32 device tensor."""
    import numpy as np
    flat = np.concatenate([np.asarray(params[k], dtype=np.float64).ravel() for k in GNN_NAMES])
    return torch.tensor(flat, dtype=torch.float32, device=device)


def gnn_unpack(flat: torch.Tensor, width: int = 32, nin: int = 4) -> dict:
    import numpy as np
    v = flat.detach().double().cpu().numpy()
    w = width
    shp = {"Ws1": (nin, w), "Wm1": (nin, w), "b1": (w,), "Ws2": (w, w), "Wm2": (w, w),
           "b2": (w,), "Ws3": (w, w), "Wm3": (w, w), "b3": (w,), "wo": (w,)}
    out, at = {}, 0
    for k in GNN_NAMES:
        size = int(np.prod(shp[k]))
        out[k] = v[at:at + size].reshape(shp[k])
        at += size
    return out


class GnnGraph:
    """Prepared per-matrix data for the learned preconditioner."""

    def __init__(self, A: DeviceCSR, width: int = 32):
        self.A, self.width = A, width
        self.c = A._c()
        nbytes = int(_lib.phsvds_gnn_workspace_bytes(A.m, A.n, A.nnz, width))
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=A.rowptr.device)
        _check(_lib.phsvds_gnn_prepare(ctypes.byref(self.c), width, self.ws.data_ptr(), nbytes,
                                       _stream()), "gnn_prepare")

    def forward(self, w, r, x, theta):
        t = torch.empty(self.A.n, dtype=torch.float32, device=r.device)
        _check(_lib.phsvds_gnn_forward(ctypes.byref(self.c), self.width, self.ws.data_ptr(),
                                       self.ws.numel(), w.data_ptr(), r.data_ptr(), x.data_ptr(),
                                       float(theta), t.data_ptr(), _stream()), "gnn_forward")
        return t

    def loss_grad(self, w, r, x, theta, tstar, grad, loss, kind="target"):
        """Accumulates the sample's loss into loss (float64 [1]) and its
        gradient into grad (float64 [nweights]): kind 'target' the distance
        to tstar, 'residual' ||C t - r||^2 / ||r||^2 (tstar unused)."""
        if kind == "residual":
            _check(_lib.phsvds_gnn_residual_loss_grad(
                ctypes.byref(self.c), self.width, self.ws.data_ptr(), self.ws.numel(),
                w.data_ptr(), r.data_ptr(), x.data_ptr(), float(theta), grad.data_ptr(),
                loss.data_ptr(), _stream()), "gnn_residual_loss_grad")
            return
        _check(_lib.phsvds_gnn_loss_grad(ctypes.byref(self.c), self.width, self.ws.data_ptr(),
                                         self.ws.numel(), w.data_ptr(), r.data_ptr(),
                                         x.data_ptr(), float(theta), tstar.data_ptr(),
                                         grad.data_ptr(), loss.data_ptr(), _stream()),
               "gnn_loss_grad")


def gnn_adam(w, m, v, grad, step, lr=1e-3, grad_scale=1.0):
    _check(_lib.phsvds_gnn_adam(w.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(),
                                w.numel(), step, lr, grad_scale, _stream()), "gnn_adam")


def harvest(A: DeviceCSR, k: int, block: int = 4, every: int = 5, max_pairs: int = 64,
            tol: float = 1e-8, cg_tol: float = 1e-8, cg_maxit: int = 2000,
            shift_scale: float = 1.0, **opt_kw):
    """(R, X, T, theta) training pairs from a float64 stage-1 run (rows of
    count x n float64 device tensors); T solves the projected equation with
    C - shift_scale * theta I."""
    import numpy as np
    opts = make_opts(block=block, **opt_kw)
    nb = ctypes.c_size_t(0)
    _check(_lib.phsvds_harvest_workspace_bytes(A.m, A.n, A.nnz, k, ctypes.byref(opts),
                                               ctypes.byref(nb)), "harvest_workspace_bytes")
    dev = A.rowptr.device
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    R = torch.empty((max(max_pairs, 1), A.n), dtype=torch.float64, device=dev)
    X = torch.empty_like(R)
    T = torch.empty_like(R)
    th = (ctypes.c_double * max(max_pairs, 1))()
    cnt = ctypes.c_int(0)
    st = _Stats()
    c = A._c()
    _check(_lib.phsvds_harvest(ctypes.byref(c), k, every, max_pairs, tol, cg_tol, cg_maxit,
                               shift_scale, ctypes.byref(opts), ws.data_ptr(), ws.numel(), _stream(),
                               R.data_ptr(), X.data_ptr(), T.data_ptr(), th, ctypes.byref(cnt),
                               ctypes.byref(st)), "harvest")
    n = cnt.value
    return R[:n], X[:n], T[:n], np.array(th[:n]), st.as_dict(k)


def train_gnn(graphs, pairs, w, epochs=20, lr=1e-3, batch=16, seed=0, log=None, on_epoch=None,
              loss_kind="target"):
    """Adam on the mean loss over mini-batches of harvested pairs.

    graphs: list of GnnGraph; pairs: list of (graph index, r, x, theta, t*)
    with float32 device vectors.  ``on_epoch(epoch, w)`` sees the weights
    after every epoch.  Returns the per-epoch mean losses."""
    import numpy as np
    nw = w.numel()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    grad = torch.zeros(nw, dtype=torch.float64, device=w.device)
    loss = torch.zeros(1, dtype=torch.float64, device=w.device)
    rng = np.random.default_rng(seed)
    step = 0
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot = 0.0
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            grad.zero_()
            loss.zero_()
            for i in idx:
                gi, r, x, th, ts = pairs[i]
                graphs[gi].loss_grad(w, r, x, th, ts, grad, loss, loss_kind)
            step += 1
            gnn_adam(w, m, v, grad, step, lr, 1.0 / len(idx))
            tot += float(loss.item())
        hist.append(tot / len(pairs))
        if log:
            log(f"epoch {ep} mean loss {hist[-1]:.4f}")
        if on_epoch:
            on_epoch(ep, w)
    return hist
