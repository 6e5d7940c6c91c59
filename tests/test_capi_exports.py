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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_softmax_default_parameters_match_the_oracle():
    """The library's own defaults (no GPU needed): the paper's parameters, and an AExp polynomial equal to
    the stored L^2 projection (the one the parity tests pass to both sides) to 1e-11 on [-8, 8] (the monomial coefficients themselves are
    ill-conditioned in their top terms)."""
    import numpy as np
    from oracle import softmax as sm
    from paper_2403_14111_amd import hetal
    p = hetal.softmax_default_params()
    ref = sm.SoftmaxParams()
    assert (p.R, p.L, p.n, p.precise, p.extend, p.comp_g, p.exp_B, p.exp_degree, p.inv_R, p.inv_iters) == \
        (ref.R, ref.L, ref.n, 1, 1, ref.comp_g, ref.exp_B, ref.exp_degree, ref.inv_R, ref.inv_iters)
    x = np.linspace(-8, 8, 2001)
    mine = np.polynomial.polynomial.polyval(x, np.array(p.exp_coeffs[:p.exp_degree + 1]))
    from tests.golden_data import aexp_coeffs
    theirs = np.polynomial.polynomial.polyval(x, np.array(aexp_coeffs()))
    assert np.abs(mine / theirs - 1).max() < 1e-11
    assert all(v == 0.0 for v in p.exp_coeffs[p.exp_degree + 1:])
