"""Builds GPU contexts and keys from the same seeded randomness as tests/oracle_setup.py."""
import numpy as np

from paper_2403_14111_amd import inputs


def make_gpu(name, seed=2000, rot_steps=(), conj=True, relin=True):
    from paper_2403_14111_amd import hetal
    ctx = hetal.Context(name)
    sk = ctx.sk_create(inputs.ternary_secret(seed, ctx.n))
    keys = ctx.keys_create()
    if relin:
        a, e = inputs.switch_key_randomness(seed, inputs.key_id(0), ctx.dnum, ctx.primes, ctx.n)
        keys.gen_relin(sk, a, e)
    gal = set(ctx.galois_rot(r) for r in rot_steps)
    gal.discard(1)
    if conj:
        gal.add(ctx.galois_conj())
    for g in sorted(gal):
        a, e = inputs.switch_key_randomness(seed, inputs.key_id(1, g), ctx.dnum, ctx.primes, ctx.n)
        keys.gen_galois(sk, g, a, e)
    return ctx, sk, keys


def encrypt_slots_gpu(ctx, sk, z, level, seed=3000, index=0, scale=None):
    pt = ctx.encode(z, level, 2.0 ** 40 if scale is None else scale)
    a, e = inputs.encryption_randomness(seed, index, ctx.q[:level + 1], ctx.n)
    return ctx.encrypt(sk, pt, a, e)


def softmax_params_with(coeffs):
    """The library's default softmax parameters with the AExp polynomial replaced by `coeffs`, so that both
    implementations of a bit-exact comparison round the very same constants."""
    from paper_2403_14111_amd import hetal
    p = hetal.softmax_default_params()
    for i in range(len(p.exp_coeffs)):
        p.exp_coeffs[i] = coeffs[i] if i < len(coeffs) else 0.0
    p.exp_degree = len(coeffs) - 1
    return p
