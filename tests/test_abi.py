"""The C-ABI library loads and exports every function include/phsvds.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "phsvds.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phsvds_\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("phsvds_svds", "phsvds_spmm_f64", "phsvds_spmm_f32", "phsvds_csr_transpose",
                 "phsvds_rr_eig", "phsvds_spmm", "phsvds_spmm_ws_bytes",
                 "phsvds_workspace_bytes", "phsvds_last_error", "phsvds_version"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1408_5535_amd as P  # loads libphsvds.so after torch's HIP runtime
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert P.version().startswith("phsvds")


def test_workspace_planning_without_gpu():
    import paper_1408_5535_amd as P
    o = P.make_opts(block=4)
    small = P.workspace_bytes(2 * 16 * 17, 256, 1024, 10, o)
    big = P.workspace_bytes(2 * 512 * 513, 512 * 512, 1048576, 10, o)
    assert 0 < small < big
    with __import__("pytest").raises(RuntimeError):
        P.workspace_bytes(10, 20, 5, 2, o)  # m < n is rejected


def test_workspace_planning_limits():
    """k up to 64 (locked vectors leave the basis, p_max stays <= 64); JDQMR
    adds its work vectors; unknown second-stage methods are rejected."""
    import pytest

    import paper_1408_5535_amd as P
    m, n, nnz = 2 * 24 * 25, 576, 2304
    for k in (1, 24, 25, 64):
        assert P.workspace_bytes(m, n, nnz, k, P.make_opts(block=4)) > 0
    with pytest.raises(RuntimeError):
        P.workspace_bytes(m, n, nnz, 65, P.make_opts(block=4))
    gd = P.workspace_bytes(m, n, nnz, 10, P.make_opts(block=4, stage2_method="gdk"))
    jd = P.workspace_bytes(m, n, nnz, 10, P.make_opts(block=4, stage2_method="jdqmr"))
    assert jd >= gd + 10 * (m + n) * 8
    o = P.make_opts(block=4)
    o.stage2_method = 2
    with pytest.raises(RuntimeError):
        P.workspace_bytes(m, n, nnz, 10, o)


def test_transposed_product_workspace():
    import paper_1408_5535_amd as P
    c = P._Csr(300, 200, 3600, None, None, None)
    lib = P._lib
    assert lib.phsvds_spmm_ws_bytes(ctypes.byref(c), 0, 0) == 0
    t64 = lib.phsvds_spmm_ws_bytes(ctypes.byref(c), 1, 0)
    t32 = lib.phsvds_spmm_ws_bytes(ctypes.byref(c), 1, 1)
    # the CSR of A^T (rowptr, columns, values) at least
    assert t64 >= 201 * 8 + 3600 * 12 and t32 > t64


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and field offsets of the option, statistics and preconditioner
    structs as gcc lays them out from include/phsvds.h, against the ctypes
    mirrors the binding passes."""
    import subprocess

    import paper_1408_5535_amd as P
    checks = {"phsvds_opts": (P._Opts, ["dynamic", "max_switch", "shifts", "k0", "c_apply",
                                        "c_inverse"]),
              "phsvds_stats": (P._Stats, ["dyn_choice", "dyn_rate", "res_stage1", "inner2",
                                          "dep_cols"]),
              "phsvds_precond": (P._Precond, ["user_solve", "user_apply_B", "user_ctx"])}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "phsvds.h"', "int main(void) {"]
    for st, (_, fields) in checks.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fields:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for st, (cls, fields) in checks.items():
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fields:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)
