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

Prints one JSON line.  --gpus above 1 is refused: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

METRIC = "encrypted 128x768x10 matmuls/s at N=2^16; HRot/s; p99 latency batched"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
SEEDS = dict(data=1002, keys=2000, enc=3000)
A_ROWS, FEAT, CLASSES, C_PAD, S0, LEVEL = 128, 768, 10, 16, 128, 11
HROT_BATCH, BATCH_REPS = 64, 5


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


# ---------------------------------------------------------------- profile summaries
# rocprofv3 kernel names -> the library's timing classes (N = 2^16: every NTT pass has 256-point sub-transforms)
PROFILE_CLASSES = [
    ("ntt_pass_kernel<8, false, false, false", "ntt_fwd_strided"),
    ("modconv_kernel<8, 0,", "ks_modup"),
    ("modconv_kernel<8, 1,", "ks_moddown"),
    ("ntt_pass_kernel<8, false, true, false", "ntt_fwd_contig"),
    ("ntt_pass_kernel<8, false, true, true", "ntt_fwd_epilogue"),   # with or without the rescale's first pass
    ("ntt_pass_kernel<8, true, true, false", "ntt_inv_contig"),
    ("ntt_pass_kernel<8, true, false, false", "ntt_inv_strided"),
    ("ks_inner_kernel", "ks_inner"),
    ("modconv_kernel<8, 2,", "rescale"),
]
PROFILE_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "kernels_n16l12_matmul_step.md")


# the sources each profiled kernel class is built from
KERNEL_SOURCES = {"ntt": ("ntt.hip", "ntt_device.hpp", "ntt_fp64.hpp", "modarith.hpp", "hetal_internal.hpp"),
                  "ks": ("keyswitch.hip", "ntt_device.hpp", "ntt_fp64.hpp", "modarith.hpp", "hetal_internal.hpp"),
                  "rns": ("rns_kernels.hip", "modarith.hpp", "hetal_internal.hpp")}


def kernel_sources_digest(cls=None):
    """sha256 over the HIP sources of a kernel class (all of them for None): a recorded counter profile is only
    valid for the sources it was taken on."""
    import hashlib
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2403_14111_amd", "csrc")
    if cls is None:
        files = sorted(f for f in os.listdir(d) if f.endswith((".hip", ".hpp")))
    else:
        files = KERNEL_SOURCES["ntt" if cls.startswith("ntt_") else "ks" if cls.startswith(("ks_", "rescale")) else "rns"]
    h = hashlib.sha256()
    for f in files:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_class(name):
    for key, cls in PROFILE_CLASSES:
        if key in name:
            return cls
    return None


def timed_window(names, steps):
    """Indices of the last `steps` repetitions of the step's kernel sequence (the timed region).  The step length
    is the period p whose p-periodic suffix of the trace is longest (ties to the smaller p): multiples of the true
    period cover no more, and accidental short periods (a step ending in two equal kernels) cover less."""
    n = len(names)
    best = None
    for p in range(1, n // steps + 1):
        m = 0
        while m < n - p and names[n - 1 - m] == names[n - 1 - m - p]:
            m += 1
        span = m + p  # length of the longest p-periodic suffix
        if span >= steps * p and (best is None or span > best[0]):
            best = (span, p)
    if best is None:
        raise SystemExit("no %d-fold repeated step found in the trace" % steps)
    p = best[1]
    return n - steps * p, n, p


def read_dispatches(path, counter=None):
    import csv
    rows = list(csv.DictReader(open(path)))
    if counter is None:
        out = [(int(r["Start_Timestamp"]), r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]), 0.0) for r in rows]
    else:
        per = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            d = per.setdefault(r["Dispatch_Id"], [int(r["Start_Timestamp"]), r["Kernel_Name"],
                                                  int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                                                  int(r["Grid_Size"]), 0.0])
            d[4] += float(r["Counter_Value"])
        out = [tuple(v) for v in per.values()]
    out.sort()
    # the calibration copy closes a profile run: split it off
    assert "copyBuffer" in out[-1][1], "profile run does not end with the calibration copy"
    return out[:-1], out[-1]


def trace_summary(directory, steps, pmc_steps, bench=None):
    """Markdown summary of rocprofv3 output under `directory` (from bench.py --profile runs)."""
    import glob
    copy_kib = 256 * 1024
    trace = glob.glob(os.path.join(directory, "trace", "*kernel_trace.csv"))[0]
    disp, _ = read_dispatches(trace)
    lo, hi, per_step = timed_window([d[1] for d in disp], steps)
    agg = {}
    for t, name, dur, grid, _ in disp[lo:hi]:
        cls = profile_class(name) or (re.findall(r"(\w+)(?:<[^>]*>)?\(", name) or [name])[0][:40]
        a = agg.setdefault(cls, [0, 0.0, 0.0])
        a[0] += 1
        a[1] += dur
        if cls in ("ntt_fwd_strided", "ntt_fwd_contig", "ntt_inv_contig", "ntt_inv_strided"):
            a[2] += grid * 16 * 16.0  # plain passes: 16 residues per thread, each read and written once
    lines = ["# Kernel profile: DiagABT + DiagATB step, N=2^16, level 11 (bench workload)", "",
             "Commands (repository root; DIR is any output folder):", "",
             "    rocprofv3 --kernel-trace --stats --output-format csv -d DIR/trace -o trace -- "
             "python bench.py --profile --steps %d --warmup 2" % steps,
             "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/FETCH_SIZE -o pmc -- "
             "python bench.py --profile --steps %d --warmup 1" % pmc_steps,
             "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/WRITE_SIZE -o pmc -- "
             "python bench.py --profile --steps %d --warmup 1" % pmc_steps,
             "    rocprofv3 --pmc SQ_INSTS_VALU --output-format csv -d DIR/SQ_INSTS_VALU -o pmc -- "
             "python bench.py --profile --steps %d --warmup 1" % pmc_steps,
             ] + (["    python bench.py --steps %d --warmup 2 --no-cpu-baseline > BENCH.json" % steps] if bench else []) + [
             "    python bench.py --trace-summary DIR --steps %d --pmc-steps %d%s" % (
                 steps, pmc_steps, " --bench-json BENCH.json" if bench else ""), "",
             "The profiled runs (--profile) issue the two products as single calls on one stream, so that every "
             "step repeats kernel for kernel; the benchmark itself runs them on two streams (the line at the end).  "
             "Timed region: the last %d steps of the trace (%d kernels per step).  HBM MB/launch: FETCH_SIZE and "
             "WRITE_SIZE (KiB per dispatch) scaled by what they read for the closing plain copy, averaged over the "
             "class's launches in the counter runs' timed steps.  HBM frac: those bytes per launch over the average "
             "launch time, against 8 TB/s.  VALU frac: SQ_INSTS_VALU (wave instructions) x 64 lanes per launch over the "
             "average launch time, against 39.3 T lane-ops/s (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz)." % (
                 steps, per_step), "",
             "| kernel | launches/step | avg us | ms/step | algorithmic GB/s | HBM MB/launch (counters) | HBM frac "
             "| VALU frac |",
             "|---|---|---|---|---|---|---|---|"]
    traffic = {}
    scales = {}
    step_total = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        f = glob.glob(os.path.join(directory, counter, "*counter_collection.csv"))
        if not f:
            continue
        d, cal = read_dispatches(f[0], counter)
        scales[counter] = copy_kib / cal[4] if cal[4] > 0 else None
        plo, phi, _ = timed_window([x[1] for x in d], pmc_steps)
        for t, name, dur, grid, v in d[plo:phi]:
            step_total[counter] = step_total.get(counter, 0.0) + v * 1024.0 * scales[counter] / pmc_steps
            cls = profile_class(name)
            if cls:
                e = traffic.setdefault(cls, {}).setdefault(counter, [0, 0.0])
                e[0] += 1
                e[1] += v * 1024.0 * scales[counter]
    valu = {}
    f = glob.glob(os.path.join(directory, "SQ_INSTS_VALU", "*counter_collection.csv"))
    if f:
        d, _ = read_dispatches(f[0], "SQ_INSTS_VALU")
        plo, phi, _ = timed_window([x[1] for x in d], pmc_steps)
        for t, name, dur, grid, v in d[plo:phi]:
            cls = profile_class(name)
            if cls:
                e = valu.setdefault(cls, [0, 0.0])
                e[0] += 1
                e[1] += v
    per_launch = {}
    for cls, e in traffic.items():
        if "FETCH_SIZE" in e and "WRITE_SIZE" in e:
            per_launch[cls] = e["FETCH_SIZE"][1] / e["FETCH_SIZE"][0] + e["WRITE_SIZE"][1] / e["WRITE_SIZE"][0]
    for cls, (n, dur, byts) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:16]:
        gbs = "%.0f" % (byts / dur) if byts else ""
        avg_s = dur / n * 1e-9
        tr = "%.1f" % (per_launch[cls] / 1e6) if cls in per_launch else ""
        hf = "%.2f" % (per_launch[cls] / avg_s / (HBM_PEAK_GBS * 1e9)) if cls in per_launch else ""
        vf = "%.2f" % (valu[cls][1] / valu[cls][0] * 64 / VALU_PEAK_LANE_OPS / avg_s) if cls in valu else ""
        lines.append("| %s | %d | %.1f | %.3f | %s | %s | %s | %s |" % (
            cls, n // steps, avg_s * 1e6, dur / steps / 1e6, gbs, tr, hf, vf))
    if bench:
        b = json.load(open(bench))
        r = b["roofline"]
        dk = r["dominant_kernel"]
        k = dk["kernel"]
        lines += ["", "bench.py (HIP events on the library stream, %d steps): %.3f matmuls/s, %.3f ms/step; the step's "
                  "minimum HBM bytes (key switch inputs, outputs and keys, no key reuse) %.2f GB, i.e. %.0f GB/s = "
                  "%.3f of 8 TB/s (%.3f with key reuse); dominant kernel %s: %.2f us per launch (trace above: "
                  "%.2f us), %.0f MB per launch." % (
                      b["steps"], b["value"], b["ms_per_step"], r["alg_bytes_per_step"] / 1e9, r["achieved"],
                      r["frac"], r["key_reuse"]["frac"], k, dk["avg_launch_us"],
                      agg[k][1] / agg[k][0] / 1e3 if k in agg else float("nan"), dk["avg_bytes_per_launch"] / 1e6)]
    lines += ["", "Counter scale factors from the closing plain copy of 256 MiB each way: " +
              ", ".join("%s x%.3f" % (k, v) for k, v in scales.items() if v), "",
              "HBM bytes per step, every kernel of the timed steps (counters, scaled): %.2f GB (FETCH %.2f, WRITE "
              "%.2f)." % (sum(step_total.values()) / 1e9, step_total.get("FETCH_SIZE", 0) / 1e9,
                          step_total.get("WRITE_SIZE", 0) / 1e9), "",
              "traffic_json: " + json.dumps({"bytes_per_launch": {k: round(v) for k, v in per_launch.items()},
                                             "bytes_per_step": round(sum(step_total.values())) if len(step_total) == 2
                                             else None,
                                             "sources_sha256_all": kernel_sources_digest(),
                                             "avg_us": {k: round(a[1] / a[0] / 1e3, 2) for k, a in agg.items()
                                                        if k in dict(PROFILE_CLASSES).values()},
                                             "sources_sha256": {k: kernel_sources_digest(k) for k in per_launch}})]
    return "\n".join(lines)


def recorded_traffic(cls):
    """HBM bytes per launch of class `cls` from the committed counter profile, if taken on these sources."""
    try:
        with open(PROFILE_FILE) as fh:
            for line in fh:
                if line.startswith("traffic_json: "):
                    rec = json.loads(line[len("traffic_json: "):])
                    digests = rec.get("sources_sha256")
                    if isinstance(digests, dict) and digests.get(cls) == kernel_sources_digest(cls):
                        return rec["bytes_per_launch"].get(cls)
    except OSError:
        pass
    return None


def recorded_step_traffic():
    """HBM bytes per step (every kernel of the step, counters) from the committed profile, if taken on these
    sources."""
    try:
        with open(PROFILE_FILE) as fh:
            for line in fh:
                if line.startswith("traffic_json: "):
                    rec = json.loads(line[len("traffic_json: "):])
                    if rec.get("sources_sha256_all") == kernel_sources_digest() and "bytes_per_step" in rec:
                        return rec["bytes_per_step"]
    except OSError:
        pass
    return None


def step_algorithmic_bytes(ctx, items, key_reads):
    """The method's minimum HBM bytes for the key switches the step ran: each key switch at level l reads its
    input and writes its output (2 (l + 1) limbs each) and reads a key of 2 beta (l + 1 + K) limbs (beta digits of
    alpha primes, K special primes).  Without key reuse every key switch reads its key; with reuse (what the
    lockstep batches do) a key is read once per batch that shares it.  Returns (no_reuse, with_reuse) bytes."""
    alpha = -(-ctx.num_q // ctx.dnum)
    io = key_all = key_once = 0
    for lv, (m, kr) in enumerate(zip(items, key_reads)):
        l = lv + 1
        key = 2 * (-(-l // alpha)) * (l + ctx.num_p)
        io += m * 4 * l
        key_all += m * key
        key_once += kr * key
    limb = ctx.n * 8
    return (io + key_all) * limb, (io + key_once) * limb


# The paper's Table 4 shapes (a, b, c) with s0 = a, its A40 seconds per call (DiagABT, DiagATB on the level(A) >=
# level(B) branch), and its corrected operation counts (Table matnum_fixed).
PAPER_SHAPES = [
    ((128, 128, 4), 0.0601, 0.0415),
    ((256, 256, 8), 0.1211, 0.1239),
    ((512, 769, 4), 0.1223, 0.3343),
    ((1024, 769, 8), 0.3710, 1.2558),
    ((2048, 769, 16), 1.2376, 4.9970),
]


def paper_shapes(reps):
    """DiagABT and both DiagATB branches at the paper's Table 4 shapes; one JSON line per shape."""
    import torch
    from paper_2403_14111_amd import hetal, inputs
    counts = {(r["a"], r["b"], r["c"]): r for r in json.load(open(os.path.join(
        os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "matnum_fixed.json")))["rows"]}
    ctx = hetal.Context("n16l12")
    sk = ctx.sk_create(inputs.ternary_secret(SEEDS["keys"], ctx.n))
    for (a, b, c), paper_abt, paper_atb in PAPER_SHAPES:
        s0 = a
        s1 = ctx.slots // s0
        log("shape %dx%dx%d: keys" % (a, b, c))
        steps = sorted(set(ctx.required_rot_steps(0, c, s0)) | set(ctx.required_rot_steps(1, c, s0)) |
                       set(ctx.required_rot_steps(2, c, s0)))
        keys = ctx.keys_create()
        ra, re_ = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(0), ctx.dnum, ctx.primes, ctx.n)
        keys.gen_relin(sk, ra, re_)
        for g in sorted(set(ctx.galois_rot(r) for r in steps) | {ctx.galois_conj()}):
            ra, re_ = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(1, g), ctx.dnum, ctx.primes, ctx.n)
            keys.gen_galois(sk, g, ra, re_)
        A = inputs.toy_matrix(SEEDS["data"] + a, a, b, 0)
        B = inputs.toy_matrix(SEEDS["data"] + a, c, b, 1)
        P = inputs.toy_matrix(SEEDS["data"] + a + 1, a, c, 0)

        def enc(mat, tiling, level, first):
            nb = int(np.prod(ctx.mat_blocks(mat.shape[0], mat.shape[1], s0, tiling, c)))
            ea, ee = enc_randomness(ctx, nb, level, first)
            return ctx.mat_encrypt(sk, mat, s0, level, 2.0 ** 40, ea, ee, tiling=tiling, c=c)

        ga = enc(A, 0, LEVEL, 0)
        gb = enc(B, 1, LEVEL, 1000)
        gp = enc(P, 2, LEVEL, 2000)
        gp_low = enc(P, 2, LEVEL - 1, 3000)
        runs = {"abt": lambda: ctx.enc_matmul_abt(keys, ga, gb, c, 1.0),
                "atb_rl": lambda: ctx.enc_matmul_atb(keys, gp, ga, c, 1.0),
                "atb_pru": lambda: ctx.enc_matmul_atb(keys, gp_low, ga, c, 1.0)}
        line = {"shape": {"a": a, "b": b, "c": c}, "s0": s0, "s1": s1, "unit": "s per call", "reps": reps}
        ops, err = {}, {}
        for name, f in runs.items():
            out = f()  # warm-up: masks are encoded once and cached
            torch.cuda.synchronize()
            ctx.reset_counters()
            f()
            torch.cuda.synchronize()
            ops[name] = ctx.counters()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                f()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            line[name + "_s"] = round(float(np.median(ts)), 5)
            res = ctx.mat_decrypt(sk, out)
            if name == "abt":
                ref = np.tile(A @ B.T, (1, s1 // c))
                err[name] = float(np.max(np.abs(res[:a, :s1] - ref)))
            else:
                ref = np.tile(P.T @ A, (s0 // c, 1))
                err[name] = float(np.max(np.abs(res[:s0, :b] - ref)))
        row = counts[(a, b, c)]
        line["ops_match_table"] = (
            {k: ops["abt"][k] for k in ("cmult", "mult", "rot")} == row["abt"]
            and {k: ops["atb_rl"][k] for k in ("cmult", "mult", "rot")} == row["atb_rl"]
            and {k: ops["atb_pru"][k] for k in ("cmult", "rot")} == row["atb_pru"])
        line["ops"] = {k: {kk: v[kk] for kk in ("rot", "conj", "mult", "cmult", "keyswitch")} for k, v in ops.items()}
        line["max_abs_err"] = err
        line["paper_a40_s"] = {"abt": paper_abt, "atb": paper_atb, "note": "A40 + HEaaN, Table 4; context only"}
        print(json.dumps(line), flush=True)
        del keys, ga, gb, gp, gp_low
        torch.cuda.empty_cache()


def uneven_requests(seed, count, per_shape):
    """`count` seeded products of uneven shapes (the survey's batching workload): rows 32..512, inner dimension
    64..1024, classes 2..100, half DiagABT (forward) and half DiagATB (gradient).  Standard encoding: s0 = 128 and
    c' = 128 for all; per-shape encoding: c' = the next power of two >= classes, s0 = the next power of two >= rows
    (at least 32 and c', at most 32768 / c' so that c' divides s1)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        rows = int(rng.integers(32, 513))
        inner = int(rng.integers(64, 1025))
        classes = int(rng.integers(2, 101))
        if per_shape:
            c = 1 << max(1, (classes - 1).bit_length())
            s0 = min(max(32, c, 1 << (rows - 1).bit_length()), 32768 // c)
        else:
            s0, c = S0, 128
        reqs.append(dict(op="abt" if i % 2 == 0 else "atb", rows=rows, inner=inner, classes=classes, s0=s0, c=c))
    return reqs


def uneven(count, per_shape, tune_reps=1):
    """Many uneven products (one JSON line): one by one, one batched call with the default schedules, the
    autotuner's schedules, and the tuned batch replayed from a HIP graph; every result the same, word for word."""
    import torch
    from paper_2403_14111_amd import hetal, inputs
    torch.cuda.set_stream(torch.cuda.Stream())   # graph capture needs a created stream
    ctx = hetal.Context("n16l12")
    sk = ctx.keygen(SEEDS["keys"])
    spec = uneven_requests(SEEDS["data"] + 7, count, per_shape)
    steps = set()
    for r in spec:
        steps |= set(ctx.required_rot_steps(0 if r["op"] == "abt" else 1, r["c"], r["s0"]))
    log("%d requests, %d rotation keys" % (len(spec), len(steps)))
    keys = ctx.keys_create()
    keys.gen_evk(sk, SEEDS["keys"], rot_steps=sorted(steps), conj=True, relin=True)
    reqs = []
    first = 0
    for n, r in enumerate(spec):
        def enc(mat, tiling):
            nonlocal first
            nb = int(np.prod(ctx.mat_blocks(mat.shape[0], mat.shape[1], r["s0"], tiling, r["c"])))
            m = ctx.mat_encrypt_seeded(sk, mat, r["s0"], LEVEL, 2.0 ** 40, SEEDS["enc"], first, tiling=tiling,
                                       c=r["c"])
            first += nb
            return m
        X = inputs.features(SEEDS["data"] + 100 + n, r["rows"], r["inner"])
        if r["op"] == "abt":
            W = inputs.weights(SEEDS["data"] + 100 + n, r["classes"], r["inner"])
            reqs.append(("abt", enc(X, 0), enc(W, 1), r["c"], 1.0))
        else:
            PY = inputs.toy_matrix(SEEDS["data"] + 100 + n, r["rows"], r["classes"], 0) * 0.1
            reqs.append(("atb", enc(PY, 2), enc(X, 0), r["c"], 1.0))
    groups = len(set((r[0], r[3], r[1].s0) for r in reqs))

    def one_by_one():
        return [ctx.enc_matmul_abt(keys, a, b, c, t) if op == "abt" else ctx.enc_matmul_atb(keys, a, b, c, t)
                for op, a, b, c, t in reqs]

    def timed(fn, reps=2):
        ts, out = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), out

    log("warm-up")
    one_by_one()
    ctx.enc_matmul_batch(keys, reqs)  # masks encoded and cached
    log("one by one")
    t_seq, seq = timed(one_by_one)
    log("batched, default schedules")
    t_bat, bat = timed(lambda: ctx.enc_matmul_batch(keys, reqs))
    log("autotuning")
    t0 = time.perf_counter()
    _, rep = ctx.autotune_batch(keys, reqs, reps=tune_reps)
    t_tuning = time.perf_counter() - t0
    t_tuned, tuned = timed(lambda: ctx.enc_matmul_batch(keys, reqs))
    log("graph of the tuned batch")
    gouts, graph = ctx.enc_matmul_batch_graph(keys, reqs)

    def replay():
        graph.launch()
        return gouts
    t_graph, _ = timed(replay)

    def same(xs, ys):
        return all(x.level == y.level and x.n_rb == y.n_rb and x.n_cb == y.n_cb and
                   torch.equal(x.buf[:x.n_rb * x.n_cb * ctx.ct_words(x.level)],
                               y.buf[:y.n_rb * y.n_cb * ctx.ct_words(y.level)]) for x, y in zip(xs, ys))
    bitexact = same(seq, bat) and same(seq, tuned) and same(seq, gouts)
    chosen = {}
    for op, a, b, c, t in reqs:
        la = min(a.level, b.level) if op == "abt" else a.level
        lb = la if op == "abt" else b.level
        chosen["%s c=%d s0=%d" % (op, c, a.s0)] = ctx.tune_get(op, c, a.s0, la, lb)
    print(json.dumps({"uneven_matmuls": count, "encoding": "per-shape s0, c'" if per_shape else "s0=128, c'=128",
                      "lockstep_groups": groups,
                      "matmuls_per_s": {"one_by_one": round(count / t_seq, 2), "batched_default": round(count / t_bat, 2),
                                        "batched_tuned": round(count / t_tuned, 2),
                                        "graph_tuned": round(count / t_graph, 2)},
                      "speedup_vs_one_by_one": {"batched_default": round(t_seq / t_bat, 3),
                                                "batched_tuned": round(t_seq / t_tuned, 3),
                                                "graph_tuned": round(t_seq / t_graph, 3)},
                      "tuned_vs_untuned": round(t_bat / t_tuned, 3), "graph_vs_eager_tuned": round(t_tuned / t_graph, 3),
                      "tuner": dict(rep, seconds=round(t_tuning, 1)), "chosen": chosen,
                      "bitexact_all_vs_one_by_one": bool(bitexact),
                      "shapes": [[r["op"], r["rows"], r["inner"], r["classes"], r["s0"], r["c"]] for r in spec]}),
          flush=True)


def serve_bench(clients, count, rates, budget_gib, lanes):
    """The request loop under Poisson arrivals (one JSON line): `clients` clients, each with its own seeded secret
    and evaluation keys (resident), four of the 64 uneven product shapes of the batching workload each (two DiagABT,
    two DiagATB, per-shape encoding), requests drawn uniformly over clients and their shapes.  Continuous batching
    on `lanes` streams with admission by free device memory; the service capacity is measured first (the 64 shapes
    in one batched call), then each offered rate is replayed: 0 stands for half the capacity (below saturation).
    p50 / p99 latency beside throughput; a sample of served results against the same products computed alone."""
    import torch
    from paper_2403_14111_amd import hetal, inputs, serving
    streams = serving.concurrent_streams(lanes)  # lanes on streams of their own, on separate hardware queues
    torch.cuda.set_stream(streams[0])
    ctx = hetal.Context("n16l12")
    spec = uneven_requests(SEEDS["data"] + 7, 4 * clients, True)
    data, owned = {}, {}
    keysets, sks = {}, {}
    first = 0
    for cl in range(clients):
        mine = spec[4 * cl:4 * cl + 4]
        steps = set()
        for r in mine:
            steps |= set(ctx.required_rot_steps(0 if r["op"] == "abt" else 1, r["c"], r["s0"]))
        sk = ctx.keygen(SEEDS["keys"] + 1 + cl)
        keys = ctx.keys_create()
        keys.gen_evk(sk, SEEDS["keys"] + 1 + cl, rot_steps=sorted(steps), conj=True, relin=True)
        sks[cl], keysets[cl] = sk, keys
        owned[cl] = []
        for j, r in enumerate(mine):
            n = 4 * cl + j
            def enc(mat, tiling):
                nonlocal first
                nb = int(np.prod(ctx.mat_blocks(mat.shape[0], mat.shape[1], r["s0"], tiling, r["c"])))
                m = ctx.mat_encrypt_seeded(sk, mat, r["s0"], LEVEL, 2.0 ** 40, SEEDS["enc"] + 1 + cl, first,
                                           tiling=tiling, c=r["c"])
                first += nb
                return m
            X = inputs.features(SEEDS["data"] + 100 + n, r["rows"], r["inner"])
            if r["op"] == "abt":
                W = inputs.weights(SEEDS["data"] + 100 + n, r["classes"], r["inner"])
                data[(cl, j)] = ("abt", enc(X, 0), enc(W, 1), r["c"])
            else:
                PY = inputs.toy_matrix(SEEDS["data"] + 100 + n, r["rows"], r["classes"], 0) * 0.1
                data[(cl, j)] = ("atb", enc(PY, 2), enc(X, 0), r["c"])
            owned[cl].append(j)
        log("client %d: %d rotation keys, 4 shapes encrypted" % (cl, len(steps)))
    torch.cuda.synchronize()
    lane_ctxs = [ctx] + [ctx.share(st) for st in streams[1:]]
    for lane in lane_ctxs:
        lane.set_two_streams(lanes == 1)
    log("warm-up on %d lanes" % lanes)
    for lane in lane_ctxs:
        with torch.cuda.stream(lane.stream):
            for cl in range(clients):
                lane.enc_matmul_batch(keysets[cl], [(op, a, b, c, 1.0) for op, a, b, c in
                                                    (data[(cl, j)] for j in owned[cl])])
    torch.cuda.synchronize()
    # capacity: every client's four shapes, one batched call per client, all lanes busy
    t0 = time.perf_counter()
    for cl in range(clients):
        lane = lane_ctxs[cl % lanes]
        with torch.cuda.stream(lane.stream):
            lane.enc_matmul_batch(keysets[cl], [(op, a, b, c, 1.0) for op, a, b, c in
                                                (data[(cl, j)] for j in owned[cl])])
    torch.cuda.synchronize()
    capacity = 4 * clients / (time.perf_counter() - t0)
    log("capacity %.1f products/s" % capacity)
    out = {"clients": clients, "lanes": lanes, "capacity_products_per_s": round(capacity, 2),
           "memory_budget_gib": budget_gib, "admission": "queue head in order while reservations fit the budget and "
           "free device memory (hipMemGetInfo + the allocator's unused cache) minus 1 GiB",
           "workload": "the 64 uneven shapes of the batching workload, 4 per client (2 DiagABT, 2 DiagATB), "
           "per-shape s0 / c', level 11, N=2^16; per-client seeded keys resident", "runs": []}
    rng = np.random.default_rng(SEEDS["data"] + 300)
    for rate in rates:
        offered = rate if rate > 0 else 0.5 * capacity
        n = int(min(count, max(64, 20.0 * min(offered, capacity))))   # about 20 s of work at most
        arrivals = serving.poisson_arrivals(rng, offered, n)
        who = rng.integers(0, clients, size=n)
        shape = rng.integers(0, 4, size=n)
        reqs = []
        for i in range(n):
            op, a, b, c = data[(int(who[i]), int(shape[i]))]
            reqs.append(serving.Request(i, int(who[i]), op, a, b, c, 1.0, arrivals[i]))
        server = serving.Server(lane_ctxs, int(budget_gib * 2 ** 30), free_memory=serving.torch_free_memory)
        for cl in range(clients):
            server.add_client(cl, keysets[cl])
        log("serving %d requests at %.1f/s" % (n, offered))
        finished = serving.serve(server, reqs)
        summary = serving.latency_summary(finished, round(offered, 2))
        sizes = [r[1] for r in server.rounds]
        same = True
        for r in finished[:: max(1, len(finished) // 6)]:
            with torch.cuda.stream(ctx.stream):
                alone = ctx.enc_matmul_batch(keysets[r.client], [(r.op, r.a, r.b, r.c, r.t)])[0]
            torch.cuda.synchronize()
            w = alone.n_rb * alone.n_cb * ctx.ct_words(alone.level)
            same = same and r.result.level == alone.level and torch.equal(r.result.buf[:w], alone.buf[:w])
        summary.update(below_saturation=bool(offered < capacity), rounds=len(sizes),
                       mean_requests_per_round=round(float(np.mean(sizes)), 2), max_requests_per_round=int(max(sizes)),
                       rounds_admitted_while_others_in_flight=sum(1 for r in server.rounds if r[3] > 0),
                       requests_per_lane=[sum(1 for r in finished if r.lane == k) for k in range(lanes)],
                       bitexact_sampled_vs_alone=bool(same))
        log("%s" % summary)
        out["runs"].append(summary)
        del finished, reqs, server
    print(json.dumps({"serving": out}), flush=True)


def softmax_bench(reps):
    """ASoftmax (App. softmax, Alg. "Row-wise softmax approximation") at the forward product's shape: the
    128 x 10 logits, classes padded to c' = 16 and tiled horizontally (s0 = 128), input at level 8 (DiagABT's
    output level), N = 2^16.  The pipeline needs ~100 levels; the key holder refreshes (decrypt and re-encrypt,
    standing in for the paper's bootstrapping), timed apart from the server's work.  Two inputs: the workload's
    own logits X W^T, and logits uniform in [-64, 64] (the extended domain).  One JSON line."""
    import torch
    from paper_2403_14111_amd import hetal, inputs
    ctx = hetal.Context("n16l12")
    sk = ctx.sk_create(inputs.ternary_secret(SEEDS["keys"], ctx.n))
    keys = ctx.keys_create()
    a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(0), ctx.dnum, ctx.primes, ctx.n)
    keys.gen_relin(sk, a, e)
    for g in sorted(set(ctx.galois_rot(r) for r in ctx.softmax_rot_steps(CLASSES, S0))):
        a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(1, g), ctx.dnum, ctx.primes, ctx.n)
        keys.gen_galois(sk, g, a, e)
    X, W, _ = workload()
    cases = {"workload_logits": X @ W.T, "uniform_64": inputs.logits(SEEDS["data"] + 400, A_ROWS, CLASSES, 64.0)}
    out = {}
    for name, M in cases.items():
        ea, ee = enc_randomness(ctx, 1, 8, 5000)
        gm = ctx.mat_encrypt(sk, M, S0, 8, 2.0 ** 40, ea, ee, tiling=2, c=C_PAD)
        spent = [0.0]
        counter = [0]

        def randomness(i):
            return inputs.refresh_randomness(SEEDS["enc"] + 77, counter[0] + i, ctx.q, ctx.n)
        base = ctx.refresher(sk, randomness)

        def timed(user, ct_ptr):
            t0 = time.perf_counter()
            rc = base(user, ct_ptr)
            torch.cuda.synchronize()
            spent[0] += time.perf_counter() - t0
            return rc
        fn = hetal.REFRESH_FN(timed)
        res, nref = ctx.softmax_approx(keys, gm, CLASSES, refresh=fn)   # warm-up: masks encoded and cached
        totals, clients = [], []
        ctx.reset_counters()
        for _ in range(reps):
            spent[0] = 0.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, nref = ctx.softmax_approx(keys, gm, CLASSES, refresh=fn)
            torch.cuda.synchronize()
            totals.append(time.perf_counter() - t0)
            clients.append(spent[0])
        cnt = ctx.counters()
        dec = ctx.mat_decrypt(sk, res)[:A_ROWS, :CLASSES]
        ex = np.exp(M - M.max(axis=1, keepdims=True))
        ex /= ex.sum(axis=1, keepdims=True)
        server = [t - c for t, c in zip(totals, clients)]
        out[name] = {"ms_per_softmax": round(1e3 * float(np.median(totals)), 2),
                     "server_ms": round(1e3 * float(np.median(server)), 2),
                     "key_holder_refresh_ms": round(1e3 * float(np.median(clients)), 2),
                     "refreshes": nref, "input_range": [round(float(M.min()), 3), round(float(M.max()), 3)],
                     "max_abs_err_vs_softmax": float(np.abs(dec - ex).max()),
                     "mean_abs_err_vs_softmax": float(np.abs(dec - ex).mean()),
                     "per_call": {k: v // reps for k, v in cnt.items() if k in ("rot", "mult", "rescale", "keyswitch")}}
        log("%s: %s" % (name, out[name]))
    print(json.dumps({"softmax_approx": out, "shape": "128 x 10 -> c'=16, s0=128, s1=256, level 8, N=2^16",
                      "reps": reps}), flush=True)


def nag_gamma(t):
    """gamma_t = (1 - lambda_t) / lambda_{t+1}, lambda_0 = 0, lambda_{t+1} = (1 + sqrt(1 + 4 lambda_t^2)) / 2."""
    lam = 0.0
    for _ in range(t):
        lam = (1.0 + np.sqrt(1.0 + 4.0 * lam * lam)) / 2.0
    return (1.0 - lam) / ((1.0 + np.sqrt(1.0 + 4.0 * lam * lam)) / 2.0)


def train_bench(steps, rows=A_ROWS, classes=CLASSES):
    """Consecutive encrypted training steps (the protocol's step 3(a): NAG with P = ASoftmax(X V^T), Sec. 3) on
    one mini-batch: X rows x 769 (768 features and the bias column), `classes` classes padded to c' (a power of
    two), s0 = rows (one block row), N = 2^16, inputs encrypted at level 11, learning rate 1 over the batch size.
    Refreshes by the key holder are timed apart.  The decrypted weights are checked against the same steps in
    FP64 with the exact softmax.  One JSON line."""
    import torch
    from paper_2403_14111_amd import hetal, inputs
    A_ROWS, CLASSES, S0 = rows, classes, rows
    C_PAD = 1
    while C_PAD < CLASSES:
        C_PAD *= 2
    ctx = hetal.Context("n16l12")
    sk = ctx.sk_create(inputs.ternary_secret(SEEDS["keys"], ctx.n))
    keys = ctx.keys_create()
    a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(0), ctx.dnum, ctx.primes, ctx.n)
    keys.gen_relin(sk, a, e)
    rot = set(ctx.softmax_rot_steps(CLASSES, S0)) | set(ctx.required_rot_steps(0, C_PAD, S0)) | \
        set(ctx.required_rot_steps(1, C_PAD, S0)) | set(ctx.required_rot_steps(2, C_PAD, S0))
    for g in sorted(set(ctx.galois_rot(r) for r in rot) | {ctx.galois_conj()}):
        a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(1, g), ctx.dnum, ctx.primes, ctx.n)
        keys.gen_galois(sk, g, a, e)
    X = np.hstack([inputs.features(SEEDS["data"], A_ROWS, FEAT), np.ones((A_ROWS, 1))])
    Y = np.eye(CLASSES)[inputs.labels(SEEDS["data"], A_ROWS, CLASSES)]
    W0 = inputs.weights(SEEDS["data"], CLASSES, FEAT + 1)

    def enc(M, tiling, first):
        nb = int(np.prod(ctx.mat_blocks(M.shape[0], M.shape[1], S0, tiling, C_PAD)))
        ea, ee = enc_randomness(ctx, nb, LEVEL, first)
        return ctx.mat_encrypt(sk, M, S0, LEVEL, 2.0 ** 40, ea, ee, tiling=tiling, c=C_PAD)
    gx, gy, gw = enc(X, 0, 6000), enc(Y, 2, 6100), enc(W0, 1, 6200)
    gv = gw
    lr = 1.0 / A_ROWS
    spent = [0.0]
    base = ctx.refresher(sk, lambda i: inputs.refresh_randomness(SEEDS["enc"] + 99, i, ctx.q, ctx.n))

    def timed(user, ct_ptr):
        t0 = time.perf_counter()
        rc = base(user, ct_ptr)
        torch.cuda.synchronize()
        spent[0] += time.perf_counter() - t0
        return rc
    fn = hetal.REFRESH_FN(timed)
    ctx.nag_step(keys, gx, gy, gw, gv, CLASSES, lr, nag_gamma(1), refresh=fn)   # warm-up: masks cached
    Wp, Vp = W0.copy(), W0.copy()
    totals, clients, nrefs = [], [], []
    for t in range(1, steps + 1):
        gamma = nag_gamma(t)
        spent[0] = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gw, gv, nref = ctx.nag_step(keys, gx, gy, gw, gv, CLASSES, lr, gamma, refresh=fn)
        torch.cuda.synchronize()
        totals.append(time.perf_counter() - t0)
        clients.append(spent[0])
        nrefs.append(nref)
        L = X @ Vp.T
        P = np.exp(L - L.max(axis=1, keepdims=True))
        P /= P.sum(axis=1, keepdims=True)
        Wn = Vp - lr * (P - Y).T @ X
        Vp, Wp = (1.0 - gamma) * Wn + gamma * Wp, Wn
        log("step %d: %.1f ms (%d refreshes)" % (t, 1e3 * totals[-1], nref))
    got = ctx.mat_decrypt(sk, gw)[:CLASSES, :FEAT + 1]

    def ce(Wm):
        L = X @ Wm.T
        L = L - L.max(axis=1, keepdims=True)
        return float(-np.mean(np.sum(Y * (L - np.log(np.exp(L).sum(axis=1, keepdims=True))), axis=1)))
    server = [t_ - c_ for t_, c_ in zip(totals, clients)]
    print(json.dumps({"train_step": {
        "ms_per_step": round(1e3 * float(np.median(totals)), 1),
        "server_ms": round(1e3 * float(np.median(server)), 1),
        "key_holder_refresh_ms": round(1e3 * float(np.median(clients)), 1),
        "refreshes_per_step": nrefs, "steps": steps,
        "max_abs_err_W_vs_fp64": float(np.abs(got - Wp).max()),
        "cross_entropy": {"start": round(ce(W0), 5), "encrypted": round(ce(got), 5), "fp64": round(ce(Wp), 5)},
        "shape": "X %d x 769 (bias column), %d classes -> c'=%d, s0=%d, s1=%d, N=2^16, inputs at level 11"
                 % (A_ROWS, CLASSES, C_PAD, S0, ctx.slots // S0), "lr": lr}}), flush=True)


def cpu_baseline(X, W, PY, gpu_coeffs):
    """The oracle (never tuned) on one full step of the same workload: one DiagABT and one DiagATB, on all
    threads; and one rotation at level 11, median of three, on all threads and on one."""
    from oracle import ckks
    from oracle import matrix as mx
    from paper_2403_14111_amd import inputs
    prm = ckks.preset("n16l12")
    sk = ckks.SecretKey(prm, inputs.ternary_secret(SEEDS["keys"], prm.n))
    ev = ckks.Evaluator(prm, sk)
    a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(0), prm.dnum, prm.all_primes, prm.n)
    ev.gen_relin_key(a, e)
    s1 = prm.slots // S0
    steps = set(mx.rotation_steps("abt", C_PAD, S0, s1)) | set(mx.rotation_steps("atb", C_PAD, S0, s1))
    for g in sorted(set(prm.galois_rot(r) for r in steps) | {prm.galois_conj}):
        a, e = inputs.switch_key_randomness(SEEDS["keys"], inputs.key_id(1, g), prm.dnum, prm.all_primes, prm.n)
        ev.gen_galois_key(g, a, e)
    Wp = np.zeros((C_PAD, FEAT))
    Wp[:CLASSES] = W
    PYp = np.zeros((A_ROWS, C_PAD))
    PYp[:, :CLASSES] = PY

    def enc(blocks, first_index):
        out = []
        for b, x in enumerate(blocks):
            pt = ckks.encode(prm, x, LEVEL, 2.0 ** 40)
            ra, re_ = inputs.encryption_randomness(SEEDS["enc"], first_index + b, prm.q[:LEVEL + 1], prm.n)
            out.append(ckks.encrypt(prm, sk, pt, ra, re_))
        return out

    xb = enc(mx.block_encode(X, S0, s1)[0], 0)
    wb = enc(mx.block_encode(mx.tile_vertical(Wp, S0), S0, s1)[0], 100)
    pb = enc(mx.block_encode(mx.tile_horizontal(PYp, s1), S0, s1)[0], 200)
    threads = ckks.LIB.orc_max_threads()
    t0 = time.perf_counter()
    out_abt = mx.diag_abt(ev, [xb], wb, C_PAD, S0, s1, 1.0)
    t_abt = time.perf_counter() - t0
    t0 = time.perf_counter()
    out_atb = mx.diag_atb(ev, [pb], [xb], C_PAD, S0, s1, 1.0)
    t_atb = time.perf_counter() - t0
    same = None
    if gpu_coeffs is not None:
        same = bool(np.array_equal(gpu_coeffs[0], out_abt[0].c) and
                    all(np.array_equal(g, o.c) for g, o in zip(gpu_coeffs[1], out_atb)))
    # one rotation at level 11, median of three, on all threads and on one
    hrot = {}
    for n in (threads, 1):
        ckks.LIB.orc_set_threads(n)
        ts = []
        for _ in range(3):
            t1 = time.perf_counter()
            ev.rot(xb[0], 1)
            ts.append(time.perf_counter() - t1)
        hrot[n] = float(np.median(ts))
    ckks.LIB.orc_set_threads(threads)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return dict(value=2.0 / (t_abt + t_atb), unit="matmuls/s", cores=threads, kind="oracle",
                sample="one full step of the workload, once: DiagABT (forward, 128x768x16) %.1f s and DiagATB "
                       "(gradient) %.1f s, N=2^16, level 11, on %d OpenMP threads" % (t_abt, t_atb, threads),
                seconds={"abt": round(t_abt, 2), "atb": round(t_atb, 2)}, cpu_model=model, nproc=os.cpu_count(),
                hrot_level11_s={"threads_%d" % threads: round(hrot[threads], 3), "one_thread": round(hrot[1], 3),
                                "of": "median of 3"}), same


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--hrot-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (e.g. under a profiler)")
    ap.add_argument("--graph", action="store_true",
                    help="replay the step as a HIP graph recorded once (hetal_enc_matmul_batch_graph)")
    ap.add_argument("--profile", action="store_true",
                    help="profiler run: warmup + timed steps + one plain copy of 256 MiB (counter calibration); "
                         "no event-timing pass, HRot loop or oracle leg")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="no GPU: summarise rocprofv3 output of --profile runs under DIR (trace/, FETCH_SIZE/, "
                         "WRITE_SIZE/) as markdown; --steps is the trace run's step count, --pmc-steps the counter "
                         "runs' one")
    ap.add_argument("--pmc-steps", type=int, default=2)
    ap.add_argument("--uneven", type=int, default=0, metavar="COUNT",
                    help="instead of the benchmark: COUNT seeded uneven products: one by one, one batched call, "
                         "autotuned, and graph-replayed (one JSON line)")
    ap.add_argument("--uneven-encoding", choices=("per-shape", "standard"), default="per-shape")
    ap.add_argument("--serve", type=int, default=0, metavar="COUNT",
                    help="instead of the benchmark: serve up to COUNT requests per offered rate, arriving as a "
                         "Poisson process (--rates per second, 0 = half the measured capacity; --clients clients, "
                         "--lanes streams, --budget-gib admission budget); one JSON line")
    ap.add_argument("--rates", default="0,200", help="comma-separated offered rates of --serve")
    ap.add_argument("--clients", type=int, default=16)
    ap.add_argument("--lanes", type=int, default=2)
    ap.add_argument("--budget-gib", type=float, default=96.0)
    ap.add_argument("--softmax", type=int, default=0, metavar="REPS",
                    help="time the softmax approximation (App. softmax) at the forward product's shape, REPS runs")
    ap.add_argument("--train-step", type=int, default=0, metavar="STEPS",
                    help="time STEPS consecutive encrypted NAG training steps (softmax included)")
    ap.add_argument("--train-shape", default="128x10", metavar="ROWSxCLASSES",
                    help="mini-batch rows and classes of --train-step (features 768 + bias), e.g. 256x100")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="instead of the benchmark: DiagABT / DiagATB (both branches) at the paper's Table 4 shapes, "
                         "one JSON line per shape (median of --steps calls)")
    ap.add_argument("--bench-json", metavar="FILE", help="with --trace-summary: a bench.py output line to compare")
    args = ap.parse_args()
    if args.trace_summary:
        print(trace_summary(args.trace_summary, args.steps, args.pmc_steps, args.bench_json))
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2403_14111_amd import hetal, inputs

    torch.cuda.set_device(0)
    if args.paper_shapes:
        paper_shapes(args.steps)
        return
    if args.uneven:
        uneven(args.uneven, args.uneven_encoding == "per-shape")
        return
    if args.softmax:
        softmax_bench(args.softmax)
        return
    if args.train_step:
        rows, classes = (int(v) for v in args.train_shape.split("x"))
        train_bench(args.train_step, rows, classes)
        return
    if args.serve:
        serve_bench(args.clients, args.serve, [float(r) for r in args.rates.split(",")], args.budget_gib,
                    args.lanes)
        return
    log("context + keys")
    if args.graph:
        torch.cuda.set_stream(torch.cuda.Stream())   # graph capture needs a created stream
    ctx = hetal.Context("n16l12")
    sk = ctx.sk_create(inputs.ternary_secret(SEEDS["keys"], ctx.n))
    t0 = time.perf_counter()
    keys, nkeys = gen_keys(ctx, sk)
    log("%d keys in %.1f s" % (nkeys, time.perf_counter() - t0))
    X, W, PY = workload()
    gx, gw, gpy = encrypt_inputs(ctx, sk, X, W, PY)
    reqs = [("abt", gx, gw, C_PAD, 1.0), ("atb", gpy, gx, C_PAD, 1.0)]
    graph = None
    if args.graph:
        log("recording the step into a HIP graph")
        graph_outs, graph = ctx.enc_matmul_batch_graph(keys, reqs)

    def eager_step():
        # one batched call: the two products are independent, and the library runs them on two streams (under a
        # profiler the single calls, one stream, so that the trace repeats kernel for kernel)
        if args.profile:
            return ctx.enc_matmul_abt(keys, gx, gw, C_PAD, 1.0), ctx.enc_matmul_atb(keys, gpy, gx, C_PAD, 1.0)
        y, g = ctx.enc_matmul_batch(keys, reqs)
        return y, g

    def step():
        if graph is not None:
            graph.launch()
            return graph_outs[0], graph_outs[1]
        return eager_step()

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
    gpu_coeffs = (ctx.ct_to_coeff(ctx.mat_block(y, 0)), [ctx.ct_to_coeff(ctx.mat_block(g, b))
                                                         for b in range(g.n_rb * g.n_cb)])

    # ---- per-kernel timing (HIP events on the library's stream), same K steps
    log("kernel timing pass")
    # with timing on the library runs the products one at a time on one stream (events per kernel); one untimed
    # step of that path first encodes the masks its context has not cached yet
    ctx.timing_enable(True)
    eager_step()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t_ev = time.perf_counter()
    for _ in range(args.steps):
        eager_step()
    torch.cuda.synchronize()
    elapsed_ev = time.perf_counter() - t_ev
    kt = ctx.timing_get()
    ctx.timing_enable(False)
    ctx.reset_counters()
    eager_step()
    torch.cuda.synchronize()
    counters_step = ctx.counters()
    ks_items, ks_reads = ctx.ks_counts()
    # the step against the method's minimum traffic: the key switches' inputs, outputs and keys over the step time
    alg_all, alg_reuse = step_algorithmic_bytes(ctx, ks_items, ks_reads)
    step_s = ms_per_step * 1e-3
    achieved = alg_all / step_s / 1e9
    traffic = recorded_step_traffic()
    # the busiest kernel class: the bytes its launches move (pipeline, not method) over its HIP-event time
    dom = max(kt, key=lambda k: kt[k]["ms"])
    d = kt[dom]
    avg_ms = d["ms"] / max(d["launches"], 1)
    avg_bytes = d["bytes"] / max(d["launches"], 1)
    dom_gbs = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roofline = dict(
        bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
        achieved=round(achieved, 1), frac=round(achieved / HBM_PEAK_GBS, 4),
        traffic=traffic,
        basis="per step: the %d key switches' minimum HBM bytes (input and output ciphertexts, one key read per key "
              "switch) over ms_per_step; traffic = every kernel's FETCH_SIZE + WRITE_SIZE per step from the "
              "committed counter profile (null if the sources changed since)" % sum(ks_items),
        alg_bytes_per_step=alg_all,
        traffic_over_alg=round(traffic / alg_all, 3) if traffic else None,
        key_switches_by_level={str(lv): m for lv, m in enumerate(ks_items) if m},
        key_reuse=dict(alg_bytes_per_step=alg_reuse, achieved=round(alg_reuse / step_s / 1e9, 1),
                       frac=round(alg_reuse / step_s / 1e9 / HBM_PEAK_GBS, 4),
                       key_reads_by_level={str(lv): m for lv, m in enumerate(ks_reads) if m}),
        dominant_kernel=dict(kernel=dom, achieved=round(dom_gbs, 1), frac=round(dom_gbs / HBM_PEAK_GBS, 4),
                             traffic=recorded_traffic(dom), avg_launch_us=round(avg_ms * 1e3, 2),
                             avg_bytes_per_launch=avg_bytes, launches_per_step=d["launches"] // args.steps,
                             note="bytes the kernel's launches read and write (the pipeline's rows) over their "
                                  "HIP-event time"))
    kernel_share = {k: dict(ms_per_step=round(v["ms"] / args.steps, 3), launches_per_step=v["launches"] // args.steps,
                            gbs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None)
                    for k, v in kt.items() if v["launches"]}

    # ---- the client's side of a step with fresh inputs, outside the timed region: the three matrices uploaded from
    # host memory, encoded and encrypted with the library's seeded sampler (PCIe included; never the `value`)
    log("client upload + encrypt")
    up_ms = []
    for rep in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.mat_encrypt_seeded(sk, X, S0, LEVEL, 2.0 ** 40, SEEDS["enc"] + 9, 0)
        ctx.mat_encrypt_seeded(sk, W, S0, LEVEL, 2.0 ** 40, SEEDS["enc"] + 9, 100, tiling=1, c=C_PAD)
        ctx.mat_encrypt_seeded(sk, PY, S0, LEVEL, 2.0 ** 40, SEEDS["enc"] + 9, 200, tiling=2, c=C_PAD)
        torch.cuda.synchronize()
        up_ms.append(1e3 * (time.perf_counter() - t0))
    upload_ms = float(np.median(up_ms))

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
    # 64 independent ciphertexts in one batched call: all by one step (one key), and each by its own step
    batch = ctx.new_ct_batch(HROT_BATCH, LEVEL)
    for b in batch:
        b.buf.copy_(ct.buf)
        b.scale = ct.scale
    out = ctx.new_ct_batch(HROT_BATCH, LEVEL)
    avail = key_steps(ctx)
    distinct = [avail[i % len(avail)] for i in range(HROT_BATCH)]
    hrot_batched = {}
    for name, steps in (("same_key", 1), ("distinct_keys", distinct)):
        ctx.hrot_batch(keys, batch, steps, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(BATCH_REPS):
            ctx.hrot_batch(keys, batch, steps, out=out)
        torch.cuda.synchronize()
        hrot_batched[name] = round(HROT_BATCH * BATCH_REPS / (time.perf_counter() - t0), 1)
    hrot_batched["distinct_key_count"] = len(set(distinct))
    del batch, out

    # ---- CPU baseline (the oracle) on one step of the same workload
    cpu = None
    bitexact = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, bitexact = cpu_baseline(X, W, PY, gpu_coeffs)

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
            "execution": "HIP graph replay" if args.graph else "batched call, two streams",
            "workload": "DiagABT <X W^T> (X 128x768, W 10x768 -> c=16) + DiagATB <(P-Y)^T X> (128x10 -> 16), "
                        "one step = both products",
            "ring": "N=2^16, 12 ciphertext primes (50+11x40 bits) + 3 special primes, dnum=4, scale 2^40",
            "level_in": LEVEL, "s0": S0, "s1": 32768 // S0, "c": C_PAD,
            "matmuls_per_step": 2,
            "arithmetic": "residues are 64-bit integers; the NTT passes compute their exact modular products in FP64, "
                          "the other kernels in 64-bit integers",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "client_upload_encrypt_ms": round(upload_ms, 3),
        "pcie_inclusive_matmuls_per_s": round(2.0 * 1e3 / (ms_per_step + upload_ms), 2),
        "hrot_per_s": round(hrot_s, 1),
        "hrot_batched_per_s": dict(hrot_batched, batch=HROT_BATCH, level=LEVEL),
        "step_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
        "step_ms_p99": round(float(np.percentile(lat_ms, 99)), 3),
        "max_abs_err": {"abt": err_y, "atb": err_g, "bound": 2.0 ** -18},
        "bitexact_vs_oracle": bitexact,
        "kernels": kernel_share,
        "timing_pass_ms_per_step": round(1e3 * elapsed_ev / args.steps, 3),
        "ops_per_step": counters_step,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
