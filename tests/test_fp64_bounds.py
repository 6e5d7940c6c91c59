"""The FP64 modular arithmetic of the NTT passes and the fused key-switch kernels, checked on the CPU against exact
integer arithmetic: tests/fp64_bounds.cpp includes the kernels' own header (csrc/ntt_fp64.hpp), built with g++,
-mfma (so that __builtin_fma is the hardware's single-rounding FMA, as on the GPU) and contraction off."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2403_14111_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_fp64_modular_arithmetic_is_exact_within_its_bounds(tmp_path):
    exe = str(tmp_path / "fp64_bounds")
    x86 = subprocess.run(["uname", "-m"], capture_output=True, text=True).stdout.strip() == "x86_64"
    flags = ["-O2", "-std=c++17", "-ffp-contract=off", "-Wno-unknown-pragmas"] + (["-mfma"] if x86 else [])
    subprocess.check_call(["g++"] + flags + ["-I" + CSRC, "-o", exe, os.path.join(HERE, "fp64_bounds.cpp")])
    r = subprocess.run([exe, "2000000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "0", r.stdout + r.stderr
