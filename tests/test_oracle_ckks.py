"""Pins of the oracle's CKKS operations (Sec. 2.2 semantics) at the toy parameters.

Each operation is checked through decryption against its slot-level meaning,
and the exact integer identities (rescale, key switching, encryption) are
checked directly on the residues.
"""
import numpy as np
import pytest

from oracle import ckks
from paper_2403_14111_amd import inputs
from tests.oracle_setup import centred, decrypt_slots, encrypt_slots, make_oracle

NOISE = 2.0 ** -19   # single-op decryption error bound at scale 2^40 in the toy ring, where
                     # q_0 (50 bits) forms a digit alone and P is one 50-bit prime


@pytest.fixture(scope="module")
def ev():
    return make_oracle("toy", rot_steps=(1, 3, -5, 256, 1000))


def test_encrypt_decrypt(ev):
    z = inputs.slot_values(10, ev.prm.slots, bound=2.0)
    for level in (0, 2, 4):
        ct = encrypt_slots(ev, z, level)
        assert ct.level == level
        assert np.max(np.abs(decrypt_slots(ev, ct) - z)) < NOISE


def test_encryption_identity(ev):
    """c0 + c1 s - m equals the error polynomial e exactly (as centred integers)."""
    prm = ev.prm
    z = inputs.slot_values(11, prm.slots)
    pt = ckks.encode(prm, z, 1, prm.scale)
    a, e = inputs.encryption_randomness(5, 0, prm.q[:2], prm.n)
    ct = ckks.encrypt(prm, ev.sk, pt, a, e)
    m = ckks.decrypt(prm, ev.sk, ct).m
    diff = ckks.sub(m, pt.m, prm.q[:2])
    for i, q in enumerate(prm.q[:2]):
        assert list(centred(diff[i], q)) == [int(v) for v in e]


@pytest.mark.parametrize("r", [1, 3, -5, 256, 1000])
def test_rotation(ev, r):
    z = inputs.slot_values(12, ev.prm.slots)
    ct = encrypt_slots(ev, z, 3)
    out = ev.rot(ct, r)
    assert out.level == 3
    assert np.max(np.abs(decrypt_slots(ev, out) - np.roll(z, -r))) < NOISE


def test_rotation_composition(ev):
    z = inputs.slot_values(13, ev.prm.slots)
    ct = encrypt_slots(ev, z, 2)
    a = ev.rot(ev.rot(ct, 1), 3)
    b = ev.rot(ct, 3)
    b = ev.rot(b, 1)
    # Different noise, same message: Lrot(Lrot(x, 1), 3) ~ Lrot(Lrot(x, 3), 1) ~ roll(x, -4)
    for x in (a, b):
        assert np.max(np.abs(decrypt_slots(ev, x) - np.roll(z, -4))) < 2 * NOISE


def test_missing_key_raises(ev):
    ct = encrypt_slots(ev, inputs.slot_values(14, ev.prm.slots), 1)
    with pytest.raises(ckks.KeyError_):
        ev.rot(ct, 2)


def test_conjugation(ev):
    z = inputs.slot_values(15, ev.prm.slots)
    ct = encrypt_slots(ev, z, 2)
    assert np.max(np.abs(decrypt_slots(ev, ev.conj(ct)) - np.conj(z))) < NOISE


def test_mult_and_rescale(ev):
    z1 = inputs.slot_values(16, ev.prm.slots, bound=2.0)
    z2 = inputs.slot_values(17, ev.prm.slots, bound=2.0)
    c1 = encrypt_slots(ev, z1, 3, index=1)
    c2 = encrypt_slots(ev, z2, 3, index=2)
    prod = ev.mult(c1, c2)
    assert prod.level == 3 and prod.scale == ev.prm.scale ** 2
    res = ev.rescale(prod)
    assert res.level == 2 and res.scale == ev.prm.scale ** 2 / ev.prm.q[3]
    assert np.max(np.abs(decrypt_slots(ev, res) - z1 * z2)) < 4 * NOISE


def test_cmult_mask_keeps_scale(ev):
    z = inputs.slot_values(18, ev.prm.slots)
    mask = (np.arange(ev.prm.slots) % 3 == 0) * (0.5 - 0.5j)
    ct = encrypt_slots(ev, z, 3)
    out = ev.rescale(ev.cmult_mask(ct, mask))
    assert out.level == 2 and abs(out.scale / ct.scale - 1) < 1e-15
    assert np.max(np.abs(decrypt_slots(ev, out) - z * mask)) < NOISE


def test_add_sub_mul_i(ev):
    z1 = inputs.slot_values(19, ev.prm.slots)
    z2 = inputs.slot_values(20, ev.prm.slots)
    c1 = encrypt_slots(ev, z1, 2, index=1)
    c2 = encrypt_slots(ev, z2, 2, index=2)
    assert np.max(np.abs(decrypt_slots(ev, ev.add(c1, c2)) - (z1 + z2))) < 2 * NOISE
    assert np.max(np.abs(decrypt_slots(ev, ev.sub(c1, c2)) - (z1 - z2))) < 2 * NOISE
    assert np.max(np.abs(decrypt_slots(ev, ev.mul_i(c1)) - 1j * z1)) < NOISE


def test_rescale_is_rounded_division(ev):
    """For each prime below the top: c_i' * q_l + [c_l]_centred == c_i (mod q_i)."""
    prm = ev.prm
    ct = encrypt_slots(ev, inputs.slot_values(21, prm.slots), 3)
    out = ev.rescale(ct)
    ql = prm.q[3]
    for p in range(2):
        top = centred(ct.c[p, 3], ql)
        for i in range(3):
            qi = prm.q[i]
            lhs = [(int(a) * ql + int(t)) % qi for a, t in zip(out.c[p, i], top)]
            assert lhs == [int(x) for x in ct.c[p, i]]


def test_mod_drop_and_level_errors(ev):
    ct = encrypt_slots(ev, inputs.slot_values(22, ev.prm.slots), 1)
    assert ev.mod_drop(ct, 0).level == 0
    with pytest.raises(ckks.LevelError):
        ev.rescale(ev.rescale(ct))
    with pytest.raises(ckks.LevelError):
        ev.mod_drop(ct, 2)


@pytest.mark.parametrize("level", [0, 2, 4])
def test_key_switch_identity(ev, level):
    """u0 + u1 s - d s' is small noise, for s' = tau_g(s) (checked on every prime)."""
    prm = ev.prm
    rng = np.random.default_rng(level)
    qs = prm.q[:level + 1]
    d = np.stack([rng.integers(0, q, size=prm.n, dtype=np.uint64) for q in qs])
    g = prm.galois_rot(3)
    u0, u1 = ckks.key_switch(prm, d, ev.rot_keys[g], g)
    s = ev.sk.limbs[:level + 1]
    sg = ckks.automorphism(ev.sk.limbs[:level + 1], qs, prm.log_n, g)
    # with ModUp before the automorphism, the switched value is tau_g(d) * tau_g(s) = tau_g(d s)
    lhs = ckks.add(u0, ckks.polymul(u1, s, qs, prm.log_n), qs)
    rhs = ckks.polymul(ckks.automorphism(d, qs, prm.log_n, g), sg, qs, prm.log_n)
    diff = ckks.sub(lhs, rhs, qs)
    for i, q in enumerate(qs):
        c = centred(diff[i], q)
        assert max(abs(int(v)) for v in c) < 2 ** 20


def test_relinearisation_identity(ev):
    prm = ev.prm
    rng = np.random.default_rng(9)
    qs = prm.q[:3]
    d = np.stack([rng.integers(0, q, size=prm.n, dtype=np.uint64) for q in qs])
    u0, u1 = ckks.key_switch(prm, d, ev.relin_key, 1)
    s = ev.sk.limbs[:3]
    lhs = ckks.add(u0, ckks.polymul(u1, s, qs, prm.log_n), qs)
    rhs = ckks.polymul(d, ckks.polymul(s, s, qs, prm.log_n), qs, prm.log_n)
    diff = ckks.sub(lhs, rhs, qs)
    for i, q in enumerate(qs):
        assert max(abs(int(v)) for v in centred(diff[i], q)) < 2 ** 20


def test_mod_down_of_a_multiple_of_p():
    """ModDown(P x) == x exactly when x is small (the conversion of a multiple of P is 0)."""
    prm = ckks.preset("n16l12")
    rng = np.random.default_rng(4)
    x = rng.integers(-1000, 1000, size=prm.n)
    level = 4
    ext = prm.q[:level + 1] + prm.p
    px = ckks.reduce_signed(x, ext, prm.log_n)
    px = ckks.mul_scalar(px, [prm.P % q for q in ext], ext, prm.log_n)
    out = ckks.mod_down(prm, px, level)
    assert np.array_equal(out, ckks.reduce_signed(x, prm.q[:level + 1], prm.log_n))


@pytest.mark.slow
def test_full_size_rotation_and_mult():
    """N = 2^16, 12 limbs: one rotation at level 11 and one Mult + rescale decrypt correctly."""
    ev = make_oracle("n16l12", rot_steps=(1,), conj=False)
    z1 = inputs.slot_values(30, ev.prm.slots)
    z2 = inputs.slot_values(31, ev.prm.slots)
    c1 = encrypt_slots(ev, z1, 11, index=1)
    c2 = encrypt_slots(ev, z2, 11, index=2)
    r = ev.rot(c1, 1)
    assert np.max(np.abs(decrypt_slots(ev, r) - np.roll(z1, -1))) < 2.0 ** -20
    m = ev.rescale(ev.mult(c1, c2))
    assert np.max(np.abs(decrypt_slots(ev, m) - z1 * z2)) < 2.0 ** -20
