"""GPU parity on modulus chains beyond the presets, every word against the oracle:
  * 49- and 50-bit primes only (N = 2^12): every row takes the reducing FP64 butterflies;
  * 30-bit ciphertext primes: the lazy butterflies at small moduli;
  * four-prime digits with four special primes: four-term ModUp and ModDown sums;
  * N = 2^13 and 2^15: 5- and 7-stage strided passes, and the basis conversions as kernels of their own."""
import sys

import numpy as np
import pytest

from oracle import ckks
from paper_2403_14111_amd import inputs
from tests.gpu_setup import encrypt_slots_gpu, make_gpu
from tests.oracle_setup import encrypt_slots, make_oracle
from tests.test_gpu_parity import same

pytestmark = pytest.mark.gpu

CHAINS = {
    "wide49": dict(log_n=12, num_q=4, num_p=2, dnum=2, q0_bits=50, q_bits=49),
    "small30": dict(log_n=12, num_q=4, num_p=2, dnum=2, q0_bits=50, q_bits=30),
    "alpha4": dict(log_n=12, num_q=8, num_p=4, dnum=2, q0_bits=50, q_bits=40),
    # other ring sizes: 5- and 7-stage strided passes, and the conversions as kernels of their own
    "n13": dict(log_n=13, num_q=3, num_p=1, dnum=3, q0_bits=50, q_bits=40),
    "n15": dict(log_n=15, num_q=4, num_p=2, dnum=2, q0_bits=50, q_bits=40),
}
STEPS = (1, -3, 1000)


def note(msg):
    print("[case] moduli " + msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", params=sorted(CHAINS))
def chain(request):
    cfg = CHAINS[request.param]
    note("%s context + keys" % request.param)
    ctx, sk, keys = make_gpu(dict(cfg), seed=2800, rot_steps=STEPS)
    ev = make_oracle(dict(cfg), seed=2800, rot_steps=STEPS)
    return request.param, ctx, sk, keys, ev


def test_primes_and_encryption(chain):
    name, ctx, sk, keys, ev = chain
    assert ctx.primes == ev.prm.all_primes
    top = ctx.max_level
    note("%s encrypt / coefficient round trip" % name)
    z = inputs.slot_values(2801, ctx.slots)
    ct = encrypt_slots_gpu(ctx, sk, z, top, seed=3800, index=0)
    ref = encrypt_slots(ev, z, top, seed=3800, index=0)
    same(ctx.ct_to_coeff(ct), ref)
    same(ctx.ct_to_coeff(ctx.ct_from_coeff(ref.c, ref.scale)), ref)


@pytest.mark.parametrize("r", STEPS)
def test_rotations_and_conjugation(chain, r):
    name, ctx, sk, keys, ev = chain
    for level in (ctx.max_level, 1):
        note("%s hrot %d level %d" % (name, r, level))
        z = inputs.slot_values(2802, ctx.slots)
        ct = encrypt_slots_gpu(ctx, sk, z, level, seed=3800, index=1)
        ref = encrypt_slots(ev, z, level, seed=3800, index=1)
        same(ctx.ct_to_coeff(ctx.hrot(keys, ct, r)), ev.rot(ref, r))
        if r == STEPS[0]:
            same(ctx.ct_to_coeff(ctx.conj(keys, ct)), ev.conj(ref))


def test_hmult_and_rescale(chain):
    name, ctx, sk, keys, ev = chain
    level = ctx.max_level
    note("%s hmult + rescale" % name)
    z1 = inputs.slot_values(2803, ctx.slots)
    z2 = inputs.slot_values(2804, ctx.slots)
    a = encrypt_slots_gpu(ctx, sk, z1, level, seed=3800, index=2)
    b = encrypt_slots_gpu(ctx, sk, z2, level, seed=3800, index=3)
    ra = encrypt_slots(ev, z1, level, seed=3800, index=2)
    rb = encrypt_slots(ev, z2, level, seed=3800, index=3)
    prod = ctx.hmult(keys, a, b)
    rprod = ev.mult(ra, rb)
    same(ctx.ct_to_coeff(prod), rprod)
    res = ctx.rescale(prod)
    rres = ev.rescale(rprod)
    same(ctx.ct_to_coeff(res), rres)
    pt = ctx.decrypt(sk, res)
    assert np.count_nonzero(ctx.pt_to_coeff(pt) != ckks.decrypt(ev.prm, ev.sk, rres).m) == 0
