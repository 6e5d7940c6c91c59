#!/usr/bin/env python
"""Benchmark of the encrypted transfer-learning layer products on one MI355X.

Workload (the encrypted forward and gradient products of one training step
of the paper's transfer-learning layer, at the 128 x 768 x 10 shape):
  forward   <X W^T>      DiagABT, X 128 x 768 (features N(0,1) clipped to
                         [-4, 4]), W 10 x 768 (uniform in [-0.05, 0.05]),
                         classes padded to c = 16;
  gradient  <(P-Y)^T X>  DiagATB, P - Y = softmax(X W^T) - onehot(labels),
                         128 x 10 padded to 16;
at N = 2^16 (32768 slots), 12 ciphertext primes + 3 special primes, dnum = 4,
scale 2^40, both inputs at level 11, block shape s0 = 128, s1 = 256.
Inputs are seeded synthetic data with the shapes of the paper's ViT / MPNet
768-dimensional features; keys, masks and ciphertexts are resident in HBM
before the timed region.  One step = one DiagABT + one DiagATB.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "encrypted 128x768x10 matmuls/s at N=2^16; HRot/s; p99 latency batched"
HBM_PEAK_GBS = 8000.0
SEEDS = dict(data=1002, keys=2000, enc=3000)
A_ROWS, FEAT, CLASSES, C_PAD, S0, LEVEL = 128, 768, 10, 16, 128, 11


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def workload():
    from paper_2403_14111_amd import inputs
    X = inputs.features(SEEDS["data"], A_ROWS, FEAT)
    W = inputs.weights(SEEDS["data"], CLASSES, FEAT)
    lab = inputs.labels(SEEDS["data"], A_ROWS, CLASSES)
    PY = inputs.softmax_minus_onehot(X @ W.T, lab, CLASSES)
    return X, W, PY


def key_steps(ctx):
    steps = set(ctx.required_rot_steps(0, C_PAD, S0)) | set(ctx.required_rot_steps(1, C_PAD, S0))
    return sorted(steps)


def gen_keys(ctx, sk):
    from paper_2403_14111_amd import inputs
    keys = ctx.keys_create()
    a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(0), ctx.dnum, ctx.primes, ctx.n)
    keys.gen_relin(sk, a, e)
    gal = sorted(set(ctx.galois_rot(r) for r in key_steps(ctx)) | {ctx.galois_conj()})
    for g in gal:
        a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(1, g), ctx.dnum, ctx.primes, ctx.n)
        keys.gen_galois(sk, g, a, e)
    return keys, len(gal) + 1


def enc_randomness(ctx, nblocks, level, first_index):
    from paper_2403_14111_amd import inputs
    r = [inputs.encryption_randomness(SEEDS["enc"], first_index + b, ctx.q[:level + 1], ctx.n) for b in range(nblocks)]
    return np.stack([x[0] for x in r]), np.stack([x[1] for x in r])


def encrypt_inputs(ctx, sk, X, W, PY):
    nx = ctx.mat_blocks(A_ROWS, FEAT, S0)[0] * ctx.mat_blocks(A_ROWS, FEAT, S0)[1]
    a, e = enc_randomness(ctx, nx, LEVEL, 0)
    gx = ctx.mat_encrypt(sk, X, S0, LEVEL, 2.0 ** 40, a, e, tiling=0)
    nw = np.prod(ctx.mat_blocks(CLASSES, FEAT, S0, 1, C_PAD))
    a, e = enc_randomness(ctx, nw, LEVEL, 100)
    gw = ctx.mat_encrypt(sk, W, S0, LEVEL, 2.0 ** 40, a, e, tiling=1, c=C_PAD)
    npy = np.prod(ctx.mat_blocks(A_ROWS, CLASSES, S0, 2, C_PAD))
    a, e = enc_randomness(ctx, npy, LEVEL, 200)
    gpy = ctx.mat_encrypt(sk, PY, S0, LEVEL, 2.0 ** 40, a, e, tiling=2, c=C_PAD)
    return gx, gw, gpy


def cpu_baseline(X, W, gpu_abt_coeffs):
    """The oracle (never tuned) on one full DiagABT of the same workload."""
    from oracle import ckks
    from oracle import matrix as mx
    from paper_2403_14111_amd import inputs
    prm = ckks.preset("n16l12")
    sk = ckks.SecretKey(prm, inputs.ternary_secret(SEEDS["keys"], prm.n))
    ev = ckks.Evaluator(prm, sk)
    a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(0), prm.dnum, prm.all_primes, prm.n)
    ev.gen_relin_key(a, e)
    s1 = prm.slots // S0
    steps = mx.rotation_steps("abt", C_PAD, S0, s1)
    for g in sorted(set(prm.galois_rot(r) for r in steps) | {prm.galois_conj}):
        a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(1, g), prm.dnum, prm.all_primes, prm.n)
        ev.gen_galois_key(g, a, e)
    Wp = np.zeros((C_PAD, FEAT))
    Wp[:CLASSES] = W

    def enc(blocks, first_index):
        out = []
        for b, x in enumerate(blocks):
            pt = ckks.encode(prm, x, LEVEL, 2.0 ** 40)
            ra, re_ = inputs.encryption_randomness(SEEDS["enc"], first_index + b, prm.q[:LEVEL + 1], prm.n)
            out.append(ckks.encrypt(prm, sk, pt, ra, re_))
        return out

    xb = enc(mx.block_encode(X, S0, s1)[0], 0)
    wb = enc(mx.block_encode(mx.tile_vertical(Wp, S0), S0, s1)[0], 100)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    out = mx.diag_abt(ev, [xb], wb, C_PAD, S0, s1, 1.0)
    dt = time.perf_counter() - t0
    same = gpu_abt_coeffs is not None and np.array_equal(gpu_abt_coeffs, out[0].c)
    return dict(value=1.0 / dt, unit="matmuls/s", cores=threads, kind="oracle",
                sample="one full DiagABT of the forward product (128x768x16, N=2^16, level 11): %.1f s on %d "
                       "OpenMP threads (%s)" % (dt, threads, os.uname().nodename),
                seconds=dt), same


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--hrot-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (e.g. under a profiler)")
    ap.add_argument("--profile", action="store_true",
                    help="profiler run: warmup + timed steps + one plain copy of 256 MiB (counter calibration); "
                         "no event-timing pass, HRot loop or oracle leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2403_14111_amd import hetal, inputs

    torch.cuda.set_device(0)
    log("context + keys")
    ctx = hetal.Context("n16l12")
    sk = ctx.sk_create(inputs.ternary_secret(SEEDS["keys"], ctx.n))
    t0 = time.perf_counter()
    keys, nkeys = gen_keys(ctx, sk)
    log("%d keys in %.1f s" % (nkeys, time.perf_counter() - t0))
    X, W, PY = workload()
    gx, gw, gpy = encrypt_inputs(ctx, sk, X, W, PY)

    def step():
        y = ctx.enc_matmul_abt(keys, gx, gw, C_PAD, 1.0)
        g = ctx.enc_matmul_atb(keys, gpy, gx, C_PAD, 1.0)
        return y, g

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: exactly K steps
    log("timed %d steps" % args.steps)
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    out = None
    for _ in range(args.steps):
        ts = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    value = 2.0 * args.steps / elapsed

    if args.profile:
        # a plain device copy of known size, to calibrate HBM byte counters against
        src = torch.empty(32 * 1024 * 1024, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "value": round(value, 3), "ms_per_step": round(ms_per_step, 3),
                          "copy_bytes_each_way": 256 * 1024 * 1024}), flush=True)
        return

    # ---- correctness of the last step against FP64
    y, g = out
    res_y = ctx.mat_decrypt(sk, y)
    ref_y = np.tile(X @ np.vstack([W, np.zeros((C_PAD - CLASSES, FEAT))]).T, (1, ctx.slots // S0 // C_PAD))
    err_y = float(np.max(np.abs(res_y[:A_ROWS, :ctx.slots // S0] - ref_y)))
    res_g = ctx.mat_decrypt(sk, g)
    PYp = np.hstack([PY, np.zeros((A_ROWS, C_PAD - CLASSES))])
    ref_g = np.tile(PYp.T @ X, (S0 // C_PAD, 1))
    err_g = float(np.max(np.abs(res_g[:S0, :FEAT] - ref_g)))
    gpu_abt_coeffs = ctx.ct_to_coeff(ctx.mat_block(y, 0))

    # ---- per-kernel timing (HIP events on the library's stream), same K steps
    log("kernel timing pass")
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t_ev = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed_ev = time.perf_counter() - t_ev
    kt = ctx.timing_get()
    ctx.timing_enable(False)
    counters_step = None
    ctx.reset_counters()
    step()
    torch.cuda.synchronize()
    counters_step = ctx.counters()
    dom = max(kt, key=lambda k: kt[k]["ms"])
    d = kt[dom]
    avg_ms = d["ms"] / max(d["launches"], 1)
    avg_bytes = d["bytes"] / max(d["launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    avg_launch_us=round(avg_ms * 1e3, 2), avg_bytes_per_launch=avg_bytes,
                    launches_per_step=d["launches"] // args.steps)
    kernel_share = {k: dict(ms_per_step=round(v["ms"] / args.steps, 3), launches_per_step=v["launches"] // args.steps,
                            gbs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None)
                    for k, v in kt.items() if v["launches"]}

    # ---- HRot/s (single rotations at level 11)
    log("hrot")
    ct = ctx.mat_block(gx, 0)
    ctx.hrot(keys, ct, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.hrot_reps):
        ctx.hrot(keys, ct, 1)
    torch.cuda.synchronize()
    hrot_s = args.hrot_reps / (time.perf_counter() - t0)

    # ---- CPU baseline (the oracle) on one DiagABT of the same workload
    cpu = None
    bitexact = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, bitexact = cpu_baseline(X, W, gpu_abt_coeffs)

    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "matmuls/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "DiagABT <X W^T> (X 128x768, W 10x768 -> c=16) + DiagATB <(P-Y)^T X> (128x10 -> 16), "
                        "one step = both products",
            "ring": "N=2^16, 12 ciphertext primes (50+11x40 bits) + 3 special primes, dnum=4, scale 2^40",
            "level_in": LEVEL, "s0": S0, "s1": 32768 // S0, "c": C_PAD,
            "matmuls_per_step": 2,
        },
        "roofline": roofline,
        "cpu_baseline": {k: v for k, v in (cpu or {}).items() if k != "seconds"} if cpu else None,
        "hrot_per_s": round(hrot_s, 1),
        "step_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
        "step_ms_p99": round(float(np.percentile(lat_ms, 99)), 3),
        "max_abs_err": {"abt": err_y, "atb": err_g, "bound": 2.0 ** -18},
        "bitexact_vs_oracle_abt": bitexact,
        "kernels": kernel_share,
        "timing_pass_ms_per_step": round(1e3 * elapsed_ev / args.steps, 3),
        "ops_per_step": counters_step,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
