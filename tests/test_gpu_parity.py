"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Every ciphertext is compared in canonical coefficient form, element by
element, and must be bit-identical to the oracle's for the same seeded inputs.
Decrypted results are also checked against FP64 within 2^-18.
"""
import sys

import numpy as np
import pytest

from oracle import ckks
from oracle import matrix as mx
from paper_2403_14111_amd import inputs
from tests.gpu_setup import encrypt_slots_gpu, make_gpu
from tests.oracle_setup import decrypt_slots, encrypt_slots, make_oracle

pytestmark = pytest.mark.gpu
TARGET = 2.0 ** -18


def note(msg):
    print("[case] " + msg, file=sys.stderr, flush=True)


TOY_STEPS = (1, 2, 3, -5, 256, 1000, 2047)


@pytest.fixture(scope="module")
def toy():
    note("toy context + keys")
    ctx, sk, keys = make_gpu("toy", rot_steps=TOY_STEPS)
    ev = make_oracle("toy", rot_steps=TOY_STEPS)
    return ctx, sk, keys, ev


def same(gpu_coeffs, oracle_ct):
    assert gpu_coeffs.shape == oracle_ct.c.shape
    diff = np.count_nonzero(gpu_coeffs != oracle_ct.c)
    assert diff == 0, "%d of %d words differ" % (diff, gpu_coeffs.size)


def test_primes_match_the_oracle(toy):
    ctx, _, _, ev = toy
    assert ctx.primes == ev.prm.all_primes
    for name in ("n16l12",):
        from paper_2403_14111_amd import hetal
        note("primes " + name)
        assert hetal.Context(name).primes == ckks.preset(name).all_primes


@pytest.mark.parametrize("level", [0, 2, 4])
@pytest.mark.parametrize("kind", ["random", "binary", "halves"])
def test_encode_bit_exact(toy, level, kind):
    ctx, _, _, ev = toy
    note("encode %s level %d" % (kind, level))
    rng = np.random.default_rng(level + 10 * len(kind))
    if kind == "random":
        z = inputs.slot_values(level, ctx.slots, bound=4.0)
        scale = 2.0 ** 40
    elif kind == "binary":
        z = rng.integers(0, 2, ctx.slots).astype(float) + 0j
        scale = float(ctx.q[level])
    else:
        z = 0.5 * rng.integers(0, 2, ctx.slots) - 0.5j * rng.integers(0, 2, ctx.slots)
        scale = float(ctx.q[level])
    pt = ctx.encode(z, level, scale)
    ref = ckks.encode(ev.prm, z, level, scale)
    got = ctx.pt_to_coeff(pt)
    assert np.count_nonzero(got != ref.m) == 0
    back = ctx.decode(pt)
    assert np.max(np.abs(back - z)) < 1e-9


def test_encode_rejects_overflow(toy):
    from paper_2403_14111_amd import hetal
    ctx = toy[0]
    with pytest.raises(hetal.HetalError) as ei:
        ctx.encode(np.full(ctx.slots, 1e30 + 0j), 1, 2.0 ** 40)
    assert ei.value.name == "E_OVERFLOW"


@pytest.mark.parametrize("level", [0, 1, 4])
def test_encrypt_decrypt_bit_exact(toy, level):
    ctx, sk, _, ev = toy
    note("encrypt level %d" % level)
    z = inputs.slot_values(20 + level, ctx.slots, bound=2.0)
    ct = encrypt_slots_gpu(ctx, sk, z, level, index=level)
    ref = encrypt_slots(ev, z, level, index=level)
    same(ctx.ct_to_coeff(ct), ref)
    pt = ctx.decrypt(sk, ct)
    ref_pt = ckks.decrypt(ev.prm, ev.sk, ref)
    assert np.count_nonzero(ctx.pt_to_coeff(pt) != ref_pt.m) == 0
    assert np.max(np.abs(ctx.decode(pt) - z)) < 1e-6


def test_coeff_round_trip(toy):
    ctx, sk, _, ev = toy
    ref = encrypt_slots(ev, inputs.slot_values(30, ctx.slots), 3, index=7)
    ct = ctx.ct_from_coeff(ref.c, ref.scale)
    same(ctx.ct_to_coeff(ct), ref)


@pytest.mark.parametrize("r", TOY_STEPS)
@pytest.mark.parametrize("level", [0, 3, 4])
def test_hrot_bit_exact(toy, r, level):
    ctx, sk, keys, ev = toy
    note("hrot r=%d level=%d" % (r, level))
    z = inputs.slot_values(40, ctx.slots)
    ct = encrypt_slots_gpu(ctx, sk, z, level, index=3)
    ref = encrypt_slots(ev, z, level, index=3)
    same(ctx.ct_to_coeff(ctx.hrot(keys, ct, r)), ev.rot(ref, r))


def test_hrot_identity_and_missing_key(toy):
    from paper_2403_14111_amd import hetal
    ctx, sk, keys, ev = toy
    z = inputs.slot_values(41, ctx.slots)
    ct = encrypt_slots_gpu(ctx, sk, z, 2, index=4)
    assert np.array_equal(ctx.ct_to_coeff(ctx.hrot(keys, ct, 0)), ctx.ct_to_coeff(ct))
    with pytest.raises(hetal.HetalError) as ei:
        ctx.hrot(keys, ct, 7)
    assert ei.value.name == "E_NO_KEY"


@pytest.mark.parametrize("layout", ["packed_buffer", "separate"])
def test_hrot_batch_bit_exact(toy, layout):
    """One batched call: mixed steps (shared and distinct keys, and the identity), against single oracle rotations."""
    from paper_2403_14111_amd import hetal
    ctx, sk, keys, ev = toy
    level = 3
    steps = [1, 1, 2, -5, 0, 2047, 1, 256]
    note("hrot_batch %s" % layout)
    zs = [inputs.slot_values(100 + i, ctx.slots) for i in range(len(steps))]
    refs = [encrypt_slots(ev, z, level, index=40 + i) for i, z in enumerate(zs)]
    if layout == "packed_buffer":
        cts = ctx.new_ct_batch(len(steps), level)
        for i, z in enumerate(zs):
            one = encrypt_slots_gpu(ctx, sk, z, level, index=40 + i)
            cts[i].buf.copy_(one.buf)
            cts[i].scale = one.scale
    else:
        cts = [encrypt_slots_gpu(ctx, sk, z, level, index=40 + i) for i, z in enumerate(zs)]
    outs = ctx.hrot_batch(keys, cts, steps)
    for out, ref, r in zip(outs, refs, steps):
        same(ctx.ct_to_coeff(out), ev.rot(ref, r) if r else ref)
        assert out.level == level
    # outputs may not overlap the inputs
    with pytest.raises(hetal.HetalError) as ei:
        ctx.hrot_batch(keys, cts, steps, out=cts)
    assert ei.value.name == "E_INVALID_ARG"


@pytest.mark.parametrize("level", [1, 4])
def test_conj_bit_exact(toy, level):
    ctx, sk, keys, ev = toy
    note("conj level %d" % level)
    z = inputs.slot_values(50, ctx.slots)
    ct = encrypt_slots_gpu(ctx, sk, z, level, index=5)
    ref = encrypt_slots(ev, z, level, index=5)
    same(ctx.ct_to_coeff(ctx.conj(keys, ct)), ev.conj(ref))


@pytest.mark.parametrize("level", [1, 2, 4])
def test_hmult_rescale_bit_exact(toy, level):
    ctx, sk, keys, ev = toy
    note("hmult level %d" % level)
    z1 = inputs.slot_values(60, ctx.slots, bound=2.0)
    z2 = inputs.slot_values(61, ctx.slots, bound=2.0)
    a = encrypt_slots_gpu(ctx, sk, z1, level, index=1)
    b = encrypt_slots_gpu(ctx, sk, z2, level, index=2)
    ra = encrypt_slots(ev, z1, level, index=1)
    rb = encrypt_slots(ev, z2, level, index=2)
    prod = ctx.hmult(keys, a, b)
    rprod = ev.mult(ra, rb)
    same(ctx.ct_to_coeff(prod), rprod)
    res = ctx.rescale(prod)
    rres = ev.rescale(rprod)
    same(ctx.ct_to_coeff(res), rres)
    assert res.level == level - 1 and abs(res.scale / rres.scale - 1) < 1e-15
    out = ctx.decode(ctx.decrypt(sk, res))
    assert np.max(np.abs(out - z1 * z2)) < 1e-5


def test_elementwise_bit_exact(toy):
    ctx, sk, keys, ev = toy
    z1 = inputs.slot_values(70, ctx.slots)
    z2 = inputs.slot_values(71, ctx.slots)
    a = encrypt_slots_gpu(ctx, sk, z1, 3, index=1)
    b = encrypt_slots_gpu(ctx, sk, z2, 3, index=2)
    ra = encrypt_slots(ev, z1, 3, index=1)
    rb = encrypt_slots(ev, z2, 3, index=2)
    same(ctx.ct_to_coeff(ctx.add(a, b)), ev.add(ra, rb))
    same(ctx.ct_to_coeff(ctx.sub(a, b)), ev.sub(ra, rb))
    same(ctx.ct_to_coeff(ctx.mul_i(a)), ev.mul_i(ra))
    same(ctx.ct_to_coeff(ctx.mod_drop(a, 1)), ev.mod_drop(ra, 1))
    mask = (np.arange(ctx.slots) % 3 == 0) * (0.5 - 0.5j)
    pt = ctx.encode(mask, 3, float(ctx.q[3]))
    same(ctx.ct_to_coeff(ctx.cmult(a, pt)), ev.cmult_mask(ra, mask))


def test_level_and_scale_errors(toy):
    from paper_2403_14111_amd import hetal
    ctx, sk, keys, ev = toy
    a = encrypt_slots_gpu(ctx, sk, inputs.slot_values(80, ctx.slots), 0, index=1)
    b = encrypt_slots_gpu(ctx, sk, inputs.slot_values(81, ctx.slots), 1, index=2)
    with pytest.raises(hetal.HetalError) as ei:
        ctx.rescale(a)
    assert ei.value.name == "E_LEVEL"
    with pytest.raises(hetal.HetalError) as ei:
        ctx.add(a, b)
    assert ei.value.name == "E_LEVEL"
    c = encrypt_slots_gpu(ctx, sk, inputs.slot_values(82, ctx.slots), 1, index=3, scale=2.0 ** 30)
    with pytest.raises(hetal.HetalError) as ei:
        ctx.add(b, c)
    assert ei.value.name == "E_SCALE"


# --------------------------------------------------------------------------
# Matrix products at the toy ring: A 16 x 32, B 8 x 32, c = 8, s0 = 16, s1 = 128
# (plus ragged, multi-block and minimum-c shapes)
# --------------------------------------------------------------------------

def toy_mats(seed=1001):
    return inputs.toy_matrix(seed, 16, 32, 0), inputs.toy_matrix(seed, 8, 32, 1)


@pytest.fixture(scope="module")
def toy_mm():
    s0, s1 = 16, 128
    steps = set()
    for c in (2, 4, 8):
        steps |= set(mx.rotation_steps("abt", c, s0, s1)) | set(mx.rotation_steps("atb", c, s0, s1, pru=True))
    steps |= set(mx.rotation_steps("abt", 8, 8, 256))
    note("toy matmul keys")
    ctx, sk, keys = make_gpu("toy", seed=2001, rot_steps=sorted(steps))
    ev = make_oracle("toy", seed=2001, rot_steps=sorted(steps))
    return ctx, sk, keys, ev


def enc_mat_gpu(ctx, sk, mat, s0, level, tiling, c, seed):
    """GPU encryption of a block matrix with the seeded randomness enc_mat_both uses (also returns the blocks)."""
    s1 = ctx.slots // s0
    if tiling == 1:
        padded = mx.tile_vertical(np.vstack([mat, np.zeros((c - mat.shape[0], mat.shape[1]))]), s0)
    elif tiling == 2:
        padded = mx.tile_horizontal(np.hstack([mat, np.zeros((mat.shape[0], c - mat.shape[1]))]), s1)
    else:
        padded = mat
    blocks = mx.block_encode(padded, s0, s1)
    nb = sum(len(r) for r in blocks)
    rand = [inputs.encryption_randomness(seed, b, ctx.q[:level + 1], ctx.n) for b in range(nb)]
    a = np.stack([r[0] for r in rand])
    e = np.stack([r[1] for r in rand])
    return ctx.mat_encrypt(sk, mat, s0, level, 2.0 ** 40, a, e, tiling=tiling, c=c), (blocks, rand)


def enc_mat_both(ctx, sk, ev, mat, s0, level, tiling, c, seed):
    s1 = ctx.slots // s0
    if tiling == 1:
        padded = mx.tile_vertical(np.vstack([mat, np.zeros((c - mat.shape[0], mat.shape[1]))]), s0)
    elif tiling == 2:
        padded = mx.tile_horizontal(np.hstack([mat, np.zeros((mat.shape[0], c - mat.shape[1]))]), s1)
    else:
        padded = mat
    blocks = mx.block_encode(padded, s0, s1)
    nb = sum(len(r) for r in blocks)
    rand = [inputs.encryption_randomness(seed, b, ctx.q[:level + 1], ctx.n) for b in range(nb)]
    a = np.stack([r[0] for r in rand])
    e = np.stack([r[1] for r in rand])
    g = ctx.mat_encrypt(sk, mat, s0, level, 2.0 ** 40, a, e, tiling=tiling, c=c)
    o = []
    b = 0
    for row in blocks:
        orow = []
        for x in row:
            pt = ckks.encode(ev.prm, x, level, 2.0 ** 40)
            orow.append(ckks.encrypt(ev.prm, ev.sk, pt, rand[b][0], rand[b][1]))
            b += 1
        o.append(orow)
    return g, o


def compare_blocks(ctx, gmat, oblocks):
    flat = [x for row in oblocks for x in row] if isinstance(oblocks[0], list) else oblocks
    assert gmat.n_rb * gmat.n_cb == len(flat)
    for b, ref in enumerate(flat):
        same(ctx.ct_to_coeff(ctx.mat_block(gmat, b)), ref)
        assert gmat.level == ref.level and abs(gmat.scale / ref.scale - 1) < 1e-12


@pytest.mark.parametrize("shape", [(16, 32, 8, 16), (13, 45, 4, 16), (40, 300, 8, 16), (16, 32, 2, 16),
                                   (16, 200, 8, 8), (16, 1152, 8, 16)],
                         ids=["base", "ragged", "multiblock", "c2", "s0_8", "wide_36_products"])
def test_diag_abt_bit_exact(toy_mm, shape):
    ctx, sk, keys, ev = toy_mm
    a_rows, b_cols, c, s0 = shape
    s1 = ctx.slots // s0
    note("abt %s" % (shape,))
    A = inputs.toy_matrix(3000 + a_rows, a_rows, b_cols, 0)
    B = inputs.toy_matrix(3000 + a_rows, min(c, 7) if c > 2 else 2, b_cols, 1)
    ga, oa = enc_mat_both(ctx, sk, ev, A, s0, 4, 0, c, seed=11)
    gb, ob = enc_mat_both(ctx, sk, ev, B, s0, 4, 1, c, seed=12)
    gout = ctx.enc_matmul_abt(keys, ga, gb, c, 1.0)
    oout = mx.diag_abt(ev, oa, ob[0], c, s0, s1, 1.0)
    compare_blocks(ctx, gout, oout)
    res = ctx.mat_decrypt(sk, gout)
    Bp = np.vstack([B, np.zeros((c - B.shape[0], b_cols))])
    ref = np.tile(A @ Bp.T, (1, s1 // c))
    err = np.max(np.abs(res[:a_rows, :s1] - ref))
    assert err < TARGET, err


@pytest.mark.parametrize("pru", [False, True])
@pytest.mark.parametrize("shape", [(16, 32, 8), (30, 150, 4), (16, 32, 2), (16, 1152, 8)],
                         ids=["base", "multiblock", "c2", "wide_36_products"])
def test_diag_atb_bit_exact(toy_mm, pru, shape):
    ctx, sk, keys, ev = toy_mm
    a_rows, b_cols, c = shape
    s0, s1 = 16, 128
    note("atb %s pru=%s" % (shape, pru))
    A = inputs.toy_matrix(4000 + a_rows, a_rows, c, 0)
    B = inputs.toy_matrix(4000 + a_rows, a_rows, b_cols, 1)
    la = 3 if pru else 4
    ga, oa = enc_mat_both(ctx, sk, ev, A, s0, la, 2, c, seed=21)
    gb, ob = enc_mat_both(ctx, sk, ev, B, s0, 4, 0, c, seed=22)
    gout = ctx.enc_matmul_atb(keys, ga, gb, c, -0.5)
    oout = mx.diag_atb(ev, oa, ob, c, s0, s1, -0.5)
    compare_blocks(ctx, gout, oout)
    res = ctx.mat_decrypt(sk, gout)
    ref = np.tile(-0.5 * A.T @ B, (s0 // c, 1))
    err = np.max(np.abs(res[:s0, :b_cols] - ref))
    assert err < TARGET, err


def test_matmul_batch_equals_single_calls(toy_mm):
    """Seven products of mixed shapes in one call: three DiagABT sharing (c, s0) with different block grids and t
    (one lockstep group), a DiagABT with another c, two DiagATB on the RotLeft branch and one on PRotUp.  Every
    output equals the single call's, word for word; one merged product is also checked against the oracle."""
    from paper_2403_14111_amd import hetal
    ctx, sk, keys, ev = toy_mm
    s0 = 16
    note("matmul batch")

    def enc(mat, level, tiling, c, seed):
        g, _ = enc_mat_gpu(ctx, sk, mat, s0, level, tiling, c, seed)
        return g

    shapes_abt = [((16, 32), (8, 32), 8, 1.0), ((40, 300), (7, 300), 8, -0.5), ((16, 1152), (6, 1152), 8, 2.0),
                  ((16, 32), (3, 32), 4, 1.0)]
    reqs = []
    for n, ((ar, ac), (br, bc_), c, t) in enumerate(shapes_abt):
        A = inputs.toy_matrix(6000 + n, ar, ac, 0)
        B = inputs.toy_matrix(6000 + n, br, bc_, 1)
        reqs.append(("abt", enc(A, 4, 0, c, 60 + n), enc(B, 4, 1, c, 70 + n), c, t))
    shapes_atb = [((16, 8), (16, 32), 4, 4, 1.0), ((30, 8), (30, 150), 4, 4, 0.5), ((16, 8), (16, 32), 3, 4, -1.0)]
    for n, ((ar, ac), (br, bc_), la, lb, t) in enumerate(shapes_atb):
        A = inputs.toy_matrix(6100 + n, ar, ac, 0)
        B = inputs.toy_matrix(6100 + n, br, bc_, 1)
        reqs.append(("atb", enc(A, la, 2, 8, 80 + n), enc(B, lb, 0, 8, 90 + n), 8, t))
    outs = ctx.enc_matmul_batch(keys, reqs)
    for (op, a, b, c, t), out in zip(reqs, outs):
        single = ctx.enc_matmul_abt(keys, a, b, c, t) if op == "abt" else ctx.enc_matmul_atb(keys, a, b, c, t)
        assert (out.n_rb, out.n_cb, out.level) == (single.n_rb, single.n_cb, single.level)
        assert out.scale == single.scale
        for blk in range(out.n_rb * out.n_cb):
            assert np.array_equal(ctx.ct_to_coeff(ctx.mat_block(out, blk)), ctx.ct_to_coeff(ctx.mat_block(single, blk)))
    # the wide request against the oracle directly
    A = inputs.toy_matrix(6002, 16, 1152, 0)
    B = inputs.toy_matrix(6002, 6, 1152, 1)
    _, oa = enc_mat_both(ctx, sk, ev, A, s0, 4, 0, 8, seed=62)
    _, ob = enc_mat_both(ctx, sk, ev, B, s0, 4, 1, 8, seed=72)
    compare_blocks(ctx, outs[2], mx.diag_abt(ev, oa, ob[0], 8, s0, ctx.slots // s0, 2.0))
    # an invalid request fails before any work
    with pytest.raises(hetal.HetalError) as ei:
        ctx.enc_matmul_batch(keys, reqs[:2] + [("abt", reqs[0][1], reqs[0][2], 6, 1.0)])
    assert ei.value.name == "E_SHAPE"


def test_matmul_batch_error_on_the_second_stream_leaves_the_context_usable():
    """A batch whose DiagATB group (run on the second stream) misses a Galois key fails with E_NO_KEY part way;
    the streams are joined all the same, and the next batch on the same context is word for word the single
    calls'."""
    from paper_2403_14111_amd import hetal
    s0, s1, c = 16, 128, 8
    note("matmul batch error on the second stream")
    ctx, sk, keys = make_gpu("toy", seed=2002, rot_steps=sorted(mx.rotation_steps("abt", c, s0, s1)))

    def enc(mat, tiling, seed):
        return enc_mat_gpu(ctx, sk, mat, s0, 4, tiling, c, seed)[0]
    A = inputs.toy_matrix(6200, 16, 32, 0)
    B = inputs.toy_matrix(6200, 8, 32, 1)
    P = inputs.toy_matrix(6201, 16, 8, 0)
    ga, gb, gp = enc(A, 0, 61), enc(B, 1, 62), enc(P, 2, 63)
    with pytest.raises(hetal.HetalError) as ei:
        ctx.enc_matmul_batch(keys, [("abt", ga, gb, c, 1.0), ("atb", gp, ga, c, 1.0)])
    assert ei.value.name == "E_NO_KEY"
    outs = ctx.enc_matmul_batch(keys, [("abt", ga, gb, c, 1.0), ("abt", ga, gb, 4, 0.5)])
    for (cc, t), out in zip(((c, 1.0), (4, 0.5)), outs):
        single = ctx.enc_matmul_abt(keys, ga, gb, cc, t)
        assert np.array_equal(ctx.ct_to_coeff(ctx.mat_block(out, 0)), ctx.ct_to_coeff(ctx.mat_block(single, 0)))


def test_matmul_shape_and_level_errors(toy_mm):
    from paper_2403_14111_amd import hetal
    ctx, sk, keys, ev = toy_mm
    A, B = toy_mats()
    ga, _ = enc_mat_both(ctx, sk, ev, A, 16, 2, 0, 8, seed=31)
    gb, _ = enc_mat_both(ctx, sk, ev, B, 16, 2, 1, 8, seed=32)
    with pytest.raises(hetal.HetalError) as ei:
        ctx.enc_matmul_abt(keys, ga, gb, 8)
    assert ei.value.name == "E_LEVEL"
    ga, _ = enc_mat_both(ctx, sk, ev, A, 16, 4, 0, 8, seed=33)
    gb, _ = enc_mat_both(ctx, sk, ev, B, 16, 4, 1, 8, seed=34)
    with pytest.raises(hetal.HetalError) as ei:
        ctx.enc_matmul_abt(keys, ga, gb, 6)
    assert ei.value.name == "E_SHAPE"


def test_required_rot_steps_match_the_oracle(toy_mm):
    ctx = toy_mm[0]
    for c in (2, 4, 8):
        assert ctx.required_rot_steps(0, c, 16) == mx.rotation_steps("abt", c, 16, 128)
        assert ctx.required_rot_steps(1, c, 16) == mx.rotation_steps("atb", c, 16, 128)
        assert ctx.required_rot_steps(2, c, 16) == mx.rotation_steps("atb", c, 16, 128, pru=True)
