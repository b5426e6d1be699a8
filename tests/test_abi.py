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
                 "phsvds_rr_eig",
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
