"""Builds oracle evaluators with keys drawn from the shared seeded inputs (test helper)."""
import numpy as np

from oracle import ckks
from paper_2403_14111_amd import inputs


def make_oracle(name, seed=2000, rot_steps=(), conj=True, relin=True):
    """name: a preset name, or a dict of ckks.Params arguments."""
    prm = ckks.Params(**name) if isinstance(name, dict) else ckks.preset(name)
    sk = ckks.SecretKey(prm, inputs.ternary_secret(seed, prm.n))
    ev = ckks.Evaluator(prm, sk)
    if relin:
        a, e = inputs.switch_key_randomness(seed, inputs.key_id(0), prm.dnum, prm.all_primes, prm.n)
        ev.gen_relin_key(a, e)
    gal = set(prm.galois_rot(r) for r in rot_steps)
    if conj:
        gal.add(prm.galois_conj)
    for g in sorted(gal):
        a, e = inputs.switch_key_randomness(seed, inputs.key_id(1, g), prm.dnum, prm.all_primes, prm.n)
        ev.gen_galois_key(g, a, e)
    return ev


def encrypt_slots(ev, z, level, seed=3000, index=0, scale=None):
    prm = ev.prm
    pt = ckks.encode(prm, z, level, prm.scale if scale is None else scale)
    a, e = inputs.encryption_randomness(seed, index, prm.q[:level + 1], prm.n)
    return ckks.encrypt(prm, ev.sk, pt, a, e)


def decrypt_slots(ev, ct):
    return ckks.decode(ev.prm, ckks.decrypt(ev.prm, ev.sk, ct))


def centred(x, q):
    x = np.asarray(x, dtype=object)
    return np.array([int(v) - q if int(v) > q // 2 else int(v) for v in x], dtype=object)
