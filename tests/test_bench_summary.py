"""bench.py's rocprofv3 summary (host logic only) on synthetic CSV files shaped like rocprofv3's output."""
import csv
import json
import os

import bench

STEP = [("void hetal::(anonymous namespace)::ntt_pass_kernel<8, false, true, true>(...)", 1000, 4096),
        ("hetal::(anonymous namespace)::ks_inner_kernel(...)", 3000, 65536),
        ("void hetal::(anonymous namespace)::ntt_pass_kernel<8, true, false, false>(...)", 500, 2048),
        ("hetal::(anonymous namespace)::add_kernel(...)", 100, 65536),
        ("hetal::(anonymous namespace)::add_kernel(...)", 100, 65536)]  # a step ending in two equal kernels
SETUP = [("hetal::(anonymous namespace)::keygen_kernel(...)", 50, 256),
         ("hetal::(anonymous namespace)::encrypt_kernel(...)", 70, 256)]
COPY = ("__amd_rocclr_copyBuffer", 200, 131072)


def write_trace(path, steps):
    rows, t = [], 0
    for name, dur, grid in SETUP + STEP * steps + [COPY]:
        rows.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + dur, "Grid_Size_X": grid,
                     "Grid_Size_Y": 1, "Grid_Size_Z": 1})
        t += dur + 10
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def write_pmc(path, counter, steps, per_kernel_kib, copy_kib):
    rows, t, d = [], 0, 0
    for name, dur, grid in SETUP + STEP * steps + [COPY]:
        val = copy_kib if name == COPY[0] else per_kernel_kib.get(name, 1.0)
        # two instances of the counter per dispatch (e.g. two dimensions), summed by the reader
        for part in (0.25, 0.75):
            rows.append({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val * part,
                         "Start_Timestamp": t, "End_Timestamp": t + dur, "Grid_Size": grid})
        t += dur + 10
        d += 1
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_summary_window_scaling_and_traffic(tmp_path):
    d = str(tmp_path)
    for sub in ("trace", "FETCH_SIZE", "WRITE_SIZE", "SQ_INSTS_VALU"):
        os.makedirs(os.path.join(d, sub))
    write_trace(os.path.join(d, "trace", "t_kernel_trace.csv"), steps=3)
    epi = STEP[0][0]
    # FETCH_SIZE reads half of the true bytes on the closing 256 MiB copy (scale x2), WRITE_SIZE all of it
    write_pmc(os.path.join(d, "FETCH_SIZE", "p_counter_collection.csv"), "FETCH_SIZE", 2, {epi: 1000.0}, 131072.0)
    write_pmc(os.path.join(d, "WRITE_SIZE", "p_counter_collection.csv"), "WRITE_SIZE", 2, {epi: 500.0}, 262144.0)
    write_pmc(os.path.join(d, "SQ_INSTS_VALU", "p_counter_collection.csv"), "SQ_INSTS_VALU", 2, {epi: 6000.0}, 1.0)
    text = bench.trace_summary(d, steps=3, pmc_steps=2)
    assert "Timed region: the last 3 steps of the trace (5 kernels per step)" in text
    rec = json.loads(text.split("traffic_json: ")[1])
    assert rec["bytes_per_launch"]["ntt_fwd_epilogue"] == (1000 * 2 + 500) * 1024
    assert rec["avg_us"]["ntt_fwd_epilogue"] == 1.0 and rec["avg_us"]["ks_inner"] == 3.0
    assert set(rec["sources_sha256"]) == set(rec["bytes_per_launch"])
    row = [l for l in text.splitlines() if l.startswith("| ntt_fwd_epilogue ")][0].split("|")
    assert row[2].strip() == "1"                                  # launches per step
    hbm = (1000 * 2 + 500) * 1024 / 1e-6 / 8e12
    assert abs(float(row[7]) - round(hbm, 2)) < 1e-9
    valu = 6000 * 64 / bench.VALU_PEAK_LANE_OPS / 1e-6
    assert abs(float(row[8]) - round(valu, 2)) < 1e-9


def test_timed_window_skips_short_accidental_periods():
    names = list("xyz") + list("abcdd") * 4
    lo, hi, p = bench.timed_window(names, 4)
    assert (lo, hi, p) == (3, len(names), 5)
    lo, hi, p = bench.timed_window(names, 2)
    assert p == 5 and lo == len(names) - 10


def test_summary_records_the_whole_step_traffic(tmp_path):
    """bytes_per_step sums every kernel of the counter runs' timed steps (not only the classified ones), scaled."""
    d = str(tmp_path)
    for sub in ("trace", "FETCH_SIZE", "WRITE_SIZE"):
        os.makedirs(os.path.join(d, sub))
    write_trace(os.path.join(d, "trace", "t_kernel_trace.csv"), steps=3)
    epi = STEP[0][0]
    write_pmc(os.path.join(d, "FETCH_SIZE", "p_counter_collection.csv"), "FETCH_SIZE", 2, {epi: 1000.0}, 131072.0)
    write_pmc(os.path.join(d, "WRITE_SIZE", "p_counter_collection.csv"), "WRITE_SIZE", 2, {epi: 500.0}, 262144.0)
    rec = json.loads(bench.trace_summary(d, steps=3, pmc_steps=2).split("traffic_json: ")[1])
    assert rec["bytes_per_step"] == ((1000 + 4) * 2 + (500 + 4) * 1) * 1024
    assert rec["sources_sha256_all"] == bench.kernel_sources_digest()


class _Ctx:
    n, num_q, num_p, dnum = 1 << 16, 12, 3, 4


def test_step_algorithmic_bytes_follow_the_key_switch_accounting():
    """One key switch at level 11 (l = 12): ciphertext in and out 4 l limbs, key 2 beta (l + K) = 2 * 4 * 15 limbs
    (60 MiB), 84 MiB in all; level 8 (l = 9): beta = 3, key 36 MiB, 54 MiB in all.  With key reuse a batch of 8
    that shares a key reads it once."""
    items = [0] * 12
    reads = [0] * 12
    items[11], reads[11] = 1, 1
    mib = 1 << 20
    assert bench.step_algorithmic_bytes(_Ctx, items, reads) == (84 * mib, 84 * mib)
    items[11], reads[11] = 0, 0
    items[8], reads[8] = 8, 1
    no_reuse, reuse = bench.step_algorithmic_bytes(_Ctx, items, reads)
    assert no_reuse == 8 * 54 * mib and reuse == 8 * 18 * mib + 36 * mib
