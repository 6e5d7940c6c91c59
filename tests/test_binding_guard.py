"""The product path has no other implementation behind it: without libhetal.so the binding refuses to import,
and the package never imports the oracle (CPU checks, in subprocesses)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2403_14111_amd")


def run(code, cwd, timeout=300):
    return subprocess.run([sys.executable, "-c", code], cwd=cwd, capture_output=True, text=True, timeout=timeout)


def test_binding_without_the_library_fails_loudly(tmp_path):
    pkg = tmp_path / "paper_2403_14111_amd"
    pkg.mkdir()
    for f in ("__init__.py", "hetal.py", "inputs.py", "serving.py"):
        shutil.copy(os.path.join(PKG, f), pkg / f)
    r = run("from paper_2403_14111_amd import hetal", str(tmp_path))
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libhetal.so is not built" in r.stderr


@pytest.mark.skipif(not os.path.exists(os.path.join(PKG, "_lib", "libhetal.so")), reason="library not built")
def test_the_package_does_not_import_the_oracle():
    code = ("import sys\n"
            "from paper_2403_14111_amd import hetal, inputs, serving\n"
            "bad = sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.'))\n"
            "assert not bad, bad\n"
            "print('ok')\n")
    r = run(code, ROOT)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr
