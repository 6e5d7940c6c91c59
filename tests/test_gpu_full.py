"""GPU parity at the full ring: N = 2^16, 12 ciphertext primes, 3 special primes, dnum = 4.

Only this ring exercises the 256-column strided NTT pass and the full hybrid
key switch (4 digits of 3 primes); every result is compared bit for bit with
the oracle in canonical coefficient form, as in the toy-ring tests.
"""
import sys

import numpy as np
import pytest

from oracle import matrix as mx
from paper_2403_14111_amd import inputs
from tests.gpu_setup import encrypt_slots_gpu, make_gpu
from tests.oracle_setup import encrypt_slots, make_oracle
from tests.test_gpu_parity import TARGET, compare_blocks, enc_mat_both, same

pytestmark = pytest.mark.gpu

S0 = 128
STEPS = (1, -3, 4096, 16383)


def note(msg):
    print("[case] full " + msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def full():
    s1 = 32768 // S0
    steps = set(STEPS) | set(mx.rotation_steps("abt", 16, S0, s1)) | set(mx.rotation_steps("atb", 16, S0, s1))
    note("context + keys (%d rotations)" % len(steps))
    ctx, sk, keys = make_gpu("n16l12", seed=2002, rot_steps=sorted(steps))
    ev = make_oracle("n16l12", seed=2002, rot_steps=sorted(steps))
    return ctx, sk, keys, ev


@pytest.mark.parametrize("level", [11, 3])
def test_full_encrypt_and_coeff_round_trip(full, level):
    ctx, sk, _, ev = full
    note("encrypt level %d" % level)
    z = inputs.slot_values(80 + level, ctx.slots)
    ref = encrypt_slots(ev, z, level, seed=3100, index=level)
    ct = encrypt_slots_gpu(ctx, sk, z, level, seed=3100, index=level)
    same(ctx.ct_to_coeff(ct), ref)
    back = ctx.ct_from_coeff(ref.c, ref.scale)
    same(ctx.ct_to_coeff(back), ref)


@pytest.mark.parametrize("r", STEPS)
@pytest.mark.parametrize("level", [11, 4])
def test_full_hrot_bit_exact(full, r, level):
    ctx, sk, keys, ev = full
    note("hrot r=%d level=%d" % (r, level))
    z = inputs.slot_values(90, ctx.slots)
    ct = encrypt_slots_gpu(ctx, sk, z, level, seed=3100, index=20)
    ref = encrypt_slots(ev, z, level, seed=3100, index=20)
    same(ctx.ct_to_coeff(ctx.hrot(keys, ct, r)), ev.rot(ref, r))
    out = ctx.decode(ctx.decrypt(sk, ctx.hrot(keys, ct, r)))
    assert np.max(np.abs(out - np.roll(z, -r))) < TARGET


def test_full_conj_bit_exact(full):
    ctx, sk, keys, ev = full
    note("conj")
    z = inputs.slot_values(91, ctx.slots)
    ct = encrypt_slots_gpu(ctx, sk, z, 11, seed=3100, index=21)
    ref = encrypt_slots(ev, z, 11, seed=3100, index=21)
    same(ctx.ct_to_coeff(ctx.conj(keys, ct)), ev.conj(ref))


@pytest.mark.parametrize("level", [11, 1])
def test_full_hmult_rescale_bit_exact(full, level):
    ctx, sk, keys, ev = full
    note("hmult level %d" % level)
    z1 = inputs.slot_values(92, ctx.slots, bound=2.0)
    z2 = inputs.slot_values(93, ctx.slots, bound=2.0)
    a = encrypt_slots_gpu(ctx, sk, z1, level, seed=3100, index=22)
    b = encrypt_slots_gpu(ctx, sk, z2, level, seed=3100, index=23)
    ra = encrypt_slots(ev, z1, level, seed=3100, index=22)
    rb = encrypt_slots(ev, z2, level, seed=3100, index=23)
    prod = ctx.hmult(keys, a, b)
    rprod = ev.mult(ra, rb)
    same(ctx.ct_to_coeff(prod), rprod)
    res = ctx.rescale(prod)
    same(ctx.ct_to_coeff(res), ev.rescale(rprod))
    out = ctx.decode(ctx.decrypt(sk, res))
    assert np.max(np.abs(out - z1 * z2)) < TARGET


def test_full_diag_abt_bit_exact(full):
    """A 24 x 200 (one ragged block), B 10 x 200 padded to c = 16."""
    ctx, sk, keys, ev = full
    s1 = ctx.slots // S0
    note("abt 24x200 . (10x200)^T")
    A = inputs.toy_matrix(5001, 24, 200, 0)
    B = inputs.toy_matrix(5001, 10, 200, 1)
    ga, oa = enc_mat_both(ctx, sk, ev, A, S0, 11, 0, 16, seed=41)
    gb, ob = enc_mat_both(ctx, sk, ev, B, S0, 11, 1, 16, seed=42)
    gout = ctx.enc_matmul_abt(keys, ga, gb, 16, 1.0)
    oout = mx.diag_abt(ev, oa, ob[0], 16, S0, s1, 1.0)
    compare_blocks(ctx, gout, oout)
    res = ctx.mat_decrypt(sk, gout)
    Bp = np.vstack([B, np.zeros((6, 200))])
    ref = np.tile(A @ Bp.T, (1, s1 // 16))
    assert np.max(np.abs(res[:24, :s1] - ref)) < TARGET


def test_full_diag_atb_bit_exact(full):
    """A 24 x 16 (the softmax-error shape), B 24 x 200."""
    ctx, sk, keys, ev = full
    s1 = ctx.slots // S0
    note("atb (24x16)^T . 24x200")
    A = inputs.toy_matrix(5002, 24, 16, 0)
    B = inputs.toy_matrix(5002, 24, 200, 1)
    ga, oa = enc_mat_both(ctx, sk, ev, A, S0, 11, 2, 16, seed=43)
    gb, ob = enc_mat_both(ctx, sk, ev, B, S0, 11, 0, 16, seed=44)
    gout = ctx.enc_matmul_atb(keys, ga, gb, 16, -0.25)
    oout = mx.diag_atb(ev, oa, ob, 16, S0, s1, -0.25)
    compare_blocks(ctx, gout, oout)
    res = ctx.mat_decrypt(sk, gout)
    ref = np.tile(-0.25 * A.T @ B, (S0 // 16, 1))
    assert np.max(np.abs(res[:S0, :200] - ref)) < TARGET
