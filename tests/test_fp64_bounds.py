"""The FP64 modular product and reduction of the NTT kernels, checked on the CPU against exact integer arithmetic
(a C copy of the two helpers, built with gcc and -mfma so that fma() is the hardware's single-rounding FMA)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_fp64_modular_arithmetic_is_exact_within_its_bounds(tmp_path):
    exe = str(tmp_path / "fp64_bounds")
    flags = ["-O2", "-mfma"] if subprocess.run(["uname", "-m"], capture_output=True, text=True).stdout.strip() == "x86_64" else ["-O2"]
    subprocess.check_call(["gcc"] + flags + ["-o", exe, os.path.join(HERE, "fp64_bounds.c"), "-lm"])
    r = subprocess.run([exe, "2000000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "0", r.stdout + r.stderr
