"""Stored inputs shared by both sides of the softmax parity tests (tests/golden/, written by scripts that call
only the oracle)."""
import json
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def aexp_coeffs():
    """AExp's degree-12 polynomial p(x / 8) (App. softmax), as stored by tests/golden/make_aexp_coeffs.py."""
    with open(os.path.join(GOLDEN, "aexp_coeffs.json")) as f:
        return [float(c) for c in json.load(f)["coeffs"]]
