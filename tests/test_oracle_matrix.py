"""Pins of the oracle's matrix layer: block encoding (App. B.1), the identities of
Prop. 1 and Prop. 2, the exact operation counts of the corrected count table,
and decrypted DiagABT / DiagATB against FP64 matrix products.
"""
import json
import os

import numpy as np
import pytest

from oracle import ckks
from oracle import matrix as mx
from oracle import slotsim
from paper_2403_14111_amd import inputs
from tests.oracle_setup import decrypt_slots, encrypt_slots, make_oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TARGET = 2.0 ** -18   # decrypted max-abs error bound at scale 2^40


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_encoding_worked_example():
    g = load("encoding_example.json")
    syms = {}
    for i, row in enumerate(g["matrix"]):
        for j, name in enumerate(row):
            syms[name] = 10 * (i + 1) + (j + 1)
    mat = np.array([[syms[x] for x in row] for row in g["matrix"]], dtype=float)
    blocks = mx.block_encode(mat, g["s0"], g["s1"])
    assert len(blocks) == 1 and len(blocks[0]) == 1
    expect = [syms[x] if isinstance(x, str) else x for x in g["slots"]]
    assert list(blocks[0][0]) == expect


def test_encoding_block_count():
    g = load("encoding_blocks.json")
    blocks = mx.block_encode(np.ones((g["rows"], g["cols"])), g["s0"], g["s1"])
    assert sum(len(r) for r in blocks) == g["blocks"]
    back = mx.block_decode(blocks, g["s0"], g["s1"])
    assert back.shape == (16, 24) and back[:13, :21].sum() == 13 * 21 and back.sum() == 13 * 21


def _sim_abt(a, b, c, s0, seed=0, t=1.0, level=12):
    s1 = 32768 // s0
    A = inputs.toy_matrix(seed, a, b, 0)
    B = inputs.toy_matrix(seed, c, b, 1)
    ev = slotsim.SimEvaluator(32768)
    Ab = [[ev.encrypt(x, level) for x in row] for row in mx.block_encode(A, s0, s1)]
    Bb = [ev.encrypt(x, level) for x in mx.block_encode(mx.tile_vertical(B, s0), s0, s1)[0]]
    out = mx.diag_abt(ev, Ab, Bb, c, s0, s1, t)
    res = mx.block_decode([[ev.decrypt(o)] for o in out], s0, s1)
    return ev, res, A, B, out


def _sim_atb(a, b, c, s0, seed=0, t=1.0, level_a=12, level_b=12):
    s1 = 32768 // s0
    A = inputs.toy_matrix(seed, a, c, 2)
    B = inputs.toy_matrix(seed, a, b, 3)
    ev = slotsim.SimEvaluator(32768)
    Ab = [[ev.encrypt(x, level_a) for x in row] for row in mx.block_encode(mx.tile_horizontal(A, s1), s0, s1)]
    Bb = [[ev.encrypt(x, level_b) for x in row] for row in mx.block_encode(B, s0, s1)]
    out = mx.diag_atb(ev, Ab, Bb, c, s0, s1, t)
    res = mx.block_decode([[ev.decrypt(o) for o in out]], s0, s1)
    return ev, res, A, B, out


@pytest.mark.parametrize("row", load("matnum_fixed.json")["rows"], ids=lambda r: "%dx%dx%d" % (r["a"], r["b"], r["c"]))
def test_operation_counts_match_the_corrected_table(row):
    a, b, c = row["a"], row["b"], row["c"]
    ev, _, _, _, out = _sim_abt(a, b, c, s0=a)
    assert {k: ev.counts.get(k, 0) for k in ("cmult", "mult", "rot")} == row["abt"]
    assert ev.counts["conj"] == len(out)
    ev, _, _, _, _ = _sim_atb(a, b, c, s0=a)
    assert {k: ev.counts.get(k, 0) for k in ("cmult", "mult", "rot")} == row["atb_rl"]
    ev, _, _, _, _ = _sim_atb(a, b, c, s0=a, level_a=11, level_b=12)
    assert {k: ev.counts.get(k, 0) for k in ("cmult", "rot")} == row["atb_pru"]
    assert ev.counts["mult"] == row["atb_rl"]["mult"]


@pytest.mark.parametrize("a,b,c,s0,t", [(128, 768, 16, 128, 1.0), (200, 300, 8, 64, -0.7), (64, 96, 4, 128, 2.0),
                                        (16, 32, 8, 16, 1.0), (256, 1024, 2, 256, 0.25)])
def test_prop1_diag_abt_equals_abt(a, b, c, s0, t):
    ev, res, A, B, out = _sim_abt(a, b, c, s0, seed=a + b, t=t)
    s1 = 32768 // s0
    ref = t * (A @ B.T)
    got = res[:a, :s1]
    assert np.max(np.abs(got - np.tile(ref, (1, s1 // c)))) < 1e-11
    assert np.max(np.abs(res.imag)) < 1e-11
    assert all(o.level == 9 for o in out)          # Mult, CS mask, M mask: three levels


@pytest.mark.parametrize("a,b,c,s0,t,lA", [(128, 768, 16, 128, 1.0, 12), (128, 768, 16, 128, 1.0, 11),
                                           (300, 200, 8, 128, -0.5, 12), (300, 200, 8, 128, 3.0, 9),
                                           (16, 32, 8, 16, 1.0, 12)])
def test_prop2_diag_atb_equals_atb(a, b, c, s0, t, lA):
    ev, res, A, B, out = _sim_atb(a, b, c, s0, seed=a * b, t=t, level_a=lA)
    ref = t * (A.T @ B)
    assert np.max(np.abs(res[:s0, :b] - np.tile(ref, (s0 // c, 1)))) < 1e-11
    assert np.max(np.abs(res.imag)) < 1e-11
    expect_level = min(lA - 1, 11) - 2 if lA < 12 else min(lA - 2, 12) - 2
    assert all(o.level == expect_level for o in out)


def test_abt_rejects_bad_shapes():
    with pytest.raises(AssertionError):
        _sim_abt(16, 32, 6, 16)
    with pytest.raises(AssertionError):
        _sim_abt(16, 32, 32, 16)


def test_depth_exhaustion_raises():
    with pytest.raises(ckks.LevelError):
        _sim_abt(16, 32, 8, 16, level=2)


# --------------------------------------------------------------------------
# Encrypted oracle (toy ring: N = 2^12, 2048 slots; s0 = 16, s1 = 128)
# --------------------------------------------------------------------------

TOY_S0, TOY_S1, TOY_C = 16, 128, 8


@pytest.fixture(scope="module")
def toy_ev():
    steps = set(mx.rotation_steps("abt", TOY_C, TOY_S0, TOY_S1)) | set(
        mx.rotation_steps("atb", TOY_C, TOY_S0, TOY_S1, pru=True))
    return make_oracle("toy", rot_steps=sorted(steps))


def test_toy_encrypted_diag_abt(toy_ev):
    ev = toy_ev
    prm = ev.prm
    A = inputs.toy_matrix(1001, 16, 32, 0)
    B = inputs.toy_matrix(1001, 8, 32, 1)
    Ab = [[encrypt_slots(ev, x, 4, index=10 + j) for j, x in enumerate(row)] for row in mx.block_encode(A, TOY_S0, TOY_S1)]
    Bb = [encrypt_slots(ev, x, 4, index=20 + j)
          for j, x in enumerate(mx.block_encode(mx.tile_vertical(B, TOY_S0), TOY_S0, TOY_S1)[0])]
    ev.reset_counts()
    out = mx.diag_abt(ev, Ab, Bb, TOY_C, TOY_S0, TOY_S1, 1.0)
    assert ev.counts["mult"] == 4 and ev.counts["rot"] == 4 + 4 * 14 and ev.counts["conj"] == 1
    assert out[0].level == 1
    res = mx.block_decode([[decrypt_slots(ev, o)] for o in out], TOY_S0, TOY_S1)
    err = np.max(np.abs(res[:16, :TOY_S1] - np.tile(A @ B.T, (1, TOY_S1 // TOY_C))))
    assert err < TARGET, err


@pytest.mark.parametrize("pru", [False, True])
def test_toy_encrypted_diag_atb(toy_ev, pru):
    ev = toy_ev
    A = inputs.toy_matrix(1002, 16, 8, 0)
    B = inputs.toy_matrix(1002, 16, 32, 1)
    la = 3 if pru else 4
    Ab = [[encrypt_slots(ev, x, la, index=30)] for x in
          [r[0] for r in mx.block_encode(mx.tile_horizontal(A, TOY_S1), TOY_S0, TOY_S1)]]
    Bb = [[encrypt_slots(ev, x, 4, index=40 + j) for j, x in enumerate(row)] for row in mx.block_encode(B, TOY_S0, TOY_S1)]
    out = mx.diag_atb(ev, Ab, Bb, TOY_C, TOY_S0, TOY_S1, -0.5)
    assert out[0].level == 0
    res = mx.block_decode([[decrypt_slots(ev, o) for o in out]], TOY_S0, TOY_S1)
    err = np.max(np.abs(res[:16, :32] - np.tile(-0.5 * A.T @ B, (TOY_S0 // TOY_C, 1))))
    assert err < TARGET, err
