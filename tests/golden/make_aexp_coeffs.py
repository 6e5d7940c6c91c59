"""Writes aexp_coeffs.json: the AExp polynomial the parity tests hand to both implementations (App. softmax: the
degree-12 least-squares approximation of e^t on [-1, 1], evaluated at x / 8).  The paper does not print it; the
oracle's L^2 projection defines it.  Run from the repository root: python tests/golden/make_aexp_coeffs.py"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import softmax as sm  # noqa: E402

coeffs = sm.exp_coeffs(12, 8)
path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "aexp_coeffs.json")
with open(path, "w") as f:
    json.dump({"source": "oracle.softmax.exp_coeffs(12, 8): L^2 projection of e^t on [-1, 1] onto degree 12, "
                         "monomial coefficients of p(x / 8)",
               "degree": 12, "B": 8, "coeffs": [repr(c) for c in coeffs]}, f, indent=1)
    f.write("\n")
print(path)
