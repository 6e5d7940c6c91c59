"""The C-ABI library loads and exports every entry point include/hetal.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hetal.h")
LIB = os.path.join(ROOT, "paper_2403_14111_amd", "_lib", "libhetal.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hetal_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hetal_encode", "hetal_encrypt", "hetal_decrypt", "hetal_hrot", "hetal_hmult", "hetal_rescale",
                     "hetal_enc_matmul_abt", "hetal_enc_matmul_atb", "hetal_keys_gen_galois", "hetal_sk_create"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_symbol():
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None:
        pytest.skip("torch missing")
    from paper_2403_14111_amd import hetal
    assert sorted(hetal.exported_symbols()) == declared_functions()
