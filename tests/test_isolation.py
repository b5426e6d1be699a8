"""The product path and the oracle are independent, and the product has no
CPU fallback (host-only checks, no GPU needed).

* No source of the package (Python or HIP) imports or includes anything
  under oracle/, and the oracle imports nothing of the package.
* Importing the package and planning a workspace loads no oracle module.
* Without its built library the package refuses to import.
"""
import os
import re
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1408_5535_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "__pycache__" in d or "_build" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_package_sources_do_not_reference_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle\b|from\s+oracle\b|#\s*include\s*[<\"][^>\"]*oracle)",
                     re.M)
    bad = [p for p in _sources(PKG, (".py", ".hip", ".hpp", ".h", ".cpp"))
           if pat.search(open(p, encoding="utf-8").read())]
    assert not bad, bad


def test_oracle_sources_do_not_reference_the_package():
    pat = re.compile(r"^\s*(import|from)\s+paper_1408_5535_amd\b", re.M)
    bad = [p for p in _sources(ORACLE, (".py", ".c", ".h"))
           if pat.search(open(p, encoding="utf-8").read())]
    assert not bad, bad


def test_importing_the_package_loads_no_oracle_module():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1408_5535_amd as P\n"
            "P.workspace_bytes(2 * 16 * 17, 256, 1024, 10, P.make_opts(block=4))\n"
            "print(sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')))\n"
            % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "[]", out.stdout


def test_package_without_its_library_refuses_to_import(tmp_path):
    dst = tmp_path / "paper_1408_5535_amd"
    dst.mkdir()
    for f in os.listdir(PKG):
        if f.endswith(".py"):
            shutil.copy(os.path.join(PKG, f), dst / f)
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n"
            "    import paper_1408_5535_amd\n"
            "except ImportError as e:\n"
            "    print('refused:', e)\n"
            "else:\n"
            "    print('imported')\n" % str(tmp_path))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "refused:" in out.stdout and "build.py" in out.stdout, out.stdout
