"""The allocation-free rotation (hetal_hrot_noalloc) against hetal_hrot, word for word, through the C ABI.

Two calls in a row on the benchmark ring (N = 2^16, 12 + 3 primes, dnum = 4): the first at the top level,
whose key switch needs 63 MiB of the 64 MiB region, the second with a smaller input (level 4).  Each output
must equal hetal_hrot's for the same input, and the device's free memory must not drop across the calls
(nothing is allocated).  Also: the toy ring, the rejection of a parameter set whose rotation needs more
than the region, and of an in-place call.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2403_14111_amd import inputs
from tests.gpu_setup import encrypt_slots_gpu, make_gpu

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] no_alloc " + msg, file=sys.stderr, flush=True)


def words(ct):
    return ct.buf[:ct.ctx.ct_words(ct.level)].cpu().numpy()


def check_pair(ctx, sk, keys, level, r, index):
    z = inputs.slot_values(500 + index, ctx.slots)
    ct = encrypt_slots_gpu(ctx, sk, z, level, seed=3500, index=index)
    ref = ctx.hrot(keys, ct, r)
    out = ctx.new_ct(level)
    out.buf.fill_(-1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.hrot_noalloc(keys, ct, r, out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (1 << 20), "device memory dropped by %d bytes" % (free0 - free1)
    assert (out.level, out.scale) == (ref.level, ref.scale)
    assert np.array_equal(words(out), words(ref))
    return out


@pytest.fixture(scope="module")
def full():
    note("n16l12 context + keys")
    return make_gpu("n16l12", seed=2050, rot_steps=(1, 5, -7), conj=False, relin=False)


def test_noalloc_full_ring_two_calls(full):
    ctx, sk, keys = full
    note("n16l12 level 11 r=5, then level 4 r=-7")
    check_pair(ctx, sk, keys, 11, 5, 0)
    check_pair(ctx, sk, keys, 4, -7, 1)
    # and once more at the top level, after the smaller call left its contents in the region
    check_pair(ctx, sk, keys, 11, 1, 2)


def test_noalloc_toy_ring_two_calls():
    note("toy level 4 r=3, then level 1 r=1")
    ctx, sk, keys = make_gpu("toy", seed=2051, rot_steps=(1, 3), conj=False, relin=False)
    check_pair(ctx, sk, keys, 4, 3, 3)
    check_pair(ctx, sk, keys, 1, 1, 4)


def test_noalloc_rejections(full):
    from paper_2403_14111_amd import hetal
    ctx, sk, keys = full
    note("rejections")
    z = inputs.slot_values(510, ctx.slots)
    ct = encrypt_slots_gpu(ctx, sk, z, 3, seed=3500, index=5)
    with pytest.raises(hetal.HetalError) as e:
        ctx.hrot_noalloc(keys, ct, 1, ct)
    assert e.value.name == "E_INVALID_ARG"
    out = ctx.new_ct(3)
    with pytest.raises(hetal.HetalError) as e:
        ctx.hrot_noalloc(keys, ct, 2, out)  # no key for 2
    assert e.value.name == "E_NO_KEY"
    # 16 + 4 primes at N = 2^16: the top-level rotation needs 84 MiB, above the 64 MiB region
    big = hetal.Context(dict(log_n=16, num_q=16, num_p=4, dnum=4, q0_bits=50, q_bits=40))
    bkeys = big.keys_create()
    bct = big.new_ct(15)
    bct.buf.zero_()
    bct.scale = 2.0 ** 40
    bout = big.new_ct(15)
    with pytest.raises(hetal.HetalError) as e:
        big.hrot_noalloc(bkeys, bct, 1, bout)
    assert e.value.name == "E_INVALID_ARG" and "scratch" in str(e.value)
