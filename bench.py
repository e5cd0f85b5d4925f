"""AFMM benchmark on one MI355X.

Workload (default): case B, n = 4096, X ~ Poisson(3) clipped to [0,255] kept
w.p. 0.3, Y ~ N(0,1) kept w.p. 0.9 (seeded, synthetic).  One step is the
strict path: the exact addition count (Section 2.2) and the strict product
(Section 2, Case-B loop), inputs resident in HBM.  The split-BF16x3 MFMA form
and the batched persistent path are timed in the same run and reported in
their own objects.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# binary32 add peak: the published 157.3 TFLOP/s fp32 vector peak counts an FMA as
# 2 flops, i.e. 128 lanes/clk/CU.  gfx950 reaches that rate with plain v_add_f32
# on VGPR operands in long straight-line runs (a probe measured 90 %).
PEAK_ADD_TFLOPS = 78.6
# one wave64 v_add_f32 per 4 cycles per SIMD (256 CU * 4 SIMD * 16 lanes * 2.4 GHz):
# the rate loops with short add runs, scalar branches and LDS traffic settle at
SINGLE_ISSUE_TADDS = 39.3
PEAK_BF16_TFLOPS = 2500.0  # dense bf16 MFMA


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    # the engine clock climbs over the first ~0.1 s of load: 3 warm-up steps
    # (5 ms) timed the n=4096 step 9 % slow, 100 steps reach the settled rate
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--n", type=int, default=4096)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-split", action="store_true")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--table1", action="store_true",
                   help="run the paper's Table 1 parameter grid (case A) instead of the benchmark")
    p.add_argument("--lowdensity", action="store_true",
                   help="run Section 2.2's low-density regime (d1*d2 = 1/n, n = 1024..8192) "
                        "instead of the benchmark")
    p.add_argument("--c5", action="store_true",
                   help="run the case-A n=16384 workload (strict vs split, sampled-row checks) "
                        "instead of the benchmark")
    p.add_argument("--copy-mb", type=int, default=0,
                   help="first run a plain device copy of this many MiB (counter calibration)")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def event_time_ms(fn, steps, stream):
    import torch
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    t1.synchronize()
    return t0.elapsed_time(t1) / steps


def per_launch_ms(fn, launches, stream):
    """Each launch between its own pair of events: (median, min) in ms."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    ev[-1][1].synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return t[len(t) // 2], t[0]


def host_info():
    """Host CPU facts for the baseline: model, logical CPUs, the CPUs this process may
    run on, and the thread count the baseline uses (a GPU's share of the box is 16)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = None
    return {"cpu_model": model, "nproc_logical": os.cpu_count(), "cpus_allowed": allowed,
            "threads_used": baseline_threads()}


def baseline_threads():
    """Threads for the CPU baseline: the CPUs this process may use, capped at 16 (the
    host-CPU share one GPU of the box comes with)."""
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return max(1, min(16, allowed))


def cpu_baseline(w, X, Y, seconds):
    """The oracle as it stands on a bounded sample of rows: one thread, then the same
    function over disjoint row ranges on the host's cores (rows are independent; the
    C oracle runs outside the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    rows_all = rng.permutation(w.n)
    # time one row, then size the single-thread sample to half the time budget
    t = time.perf_counter()
    _, adds = oracle.strict_f32(w.case, X[rows_all[:1]], Y, rows=rows_all[:1], x_rows_only=True)
    dt = time.perf_counter() - t
    per_row = max(dt, 1e-4)
    k1 = max(1, min(w.n, int(0.5 * seconds / per_row)))
    rows = rows_all[:k1]
    t = time.perf_counter()
    _, adds1 = oracle.strict_f32(w.case, X[rows], Y, rows=rows, x_rows_only=True)
    dt1 = time.perf_counter() - t
    # the same function on P threads, each a contiguous chunk of the sample
    P = baseline_threads()
    kp = max(P, min(w.n, int(0.5 * seconds * P / per_row)))
    chunks = np.array_split(rows_all[:kp], P)

    def run(ch):
        return oracle.strict_f32(w.case, X[ch], Y, rows=ch, x_rows_only=True)[1]

    t = time.perf_counter()
    with ThreadPoolExecutor(P) as ex:
        addsp = sum(ex.map(run, chunks))
    dtp = time.perf_counter() - t
    return {"value": addsp / dtp, "unit": "useful adds/s", "cores": P, "kind": "oracle",
            "host": host_info(),
            "paper_context": "Table 1, one Pentium at 1.6 GHz (Section 2.3.1): the case-A loop at "
                             "n=2000 took 53.4 s (mu'=1) to 145.9 s (mu'=7), 2.5e7 to 1.1e8 "
                             "additions/s; a different workload and machine",
            "sample": f"{kp} of {w.n} rows of the same workload over {P} threads "
                      f"({addsp} additions, {dtp:.1f} s)",
            "single_thread": {"value": adds1 / dt1, "cores": 1,
                              "sample": f"{k1} rows ({adds1} additions, {dt1:.1f} s)"}}


# the strict kernels' sources: a committed traffic measurement is used only while
# none of them has changed since the counters were taken
STRICT_SOURCES = tuple("paper_1308_2400_amd/csrc/" + f for f in (
    "common.hpp", "strict_body.hpp", "sparse_body.hpp", "strict_kernels.hpp", "strict.hip",
    "strict_part_a.hip", "strict_part_b.hip", "strict_part_c.hip", "strict_sparse.hip"))


def strict_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STRICT_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(config):
    """HBM bytes per strict launch from the committed counter runs, if they were taken
    on this kernel configuration and these kernel sources."""
    path = os.path.join(ROOT, "profiles", "rep_uniform_caseB_n4096_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != strict_source_hash() or list(d.get("kernel_config", [])) != list(config):
        return None
    return d.get("hbm_bytes_per_launch")


def bench_batched(args, stream, single_issued_frac, single_useful_per_s):
    """512 products of uneven n, density and integer range: one plan, graph replays."""
    import numpy as np
    import torch

    import gen
    import oracle
    import paper_1308_2400_amd as afmm

    dev = torch.device("cuda:0")
    ws = gen.batched_512()
    log(f"bench: generating {len(ws)} batched products")
    host = [(w.case, w.X(), w.Y()) for w in ws]
    probs = []
    issued = 0
    for case, X, Y in host:
        n = X.shape[0]
        ints = Y if case == "A" else X
        issued += int(np.maximum(ints, 0).astype(np.int64).sum()) * n
        Xd = torch.from_numpy(X).to(dev)
        Yd = torch.from_numpy(Y).to(dev)
        probs.append((case, Xd, Yd, torch.empty((n, n), dtype=torch.float32, device=dev)))
    plan = afmm.Plan(probs)
    for _ in range(min(args.warmup, 10)):  # a plan launch takes ~30 ms
        plan.launch()
    torch.cuda.synchronize()
    ms = event_time_ms(plan.launch, args.steps, stream)
    adds = sum(plan.problem_adds())
    # the same 512 products as separate single-product calls (the library's own
    # choice of kernel per product, one workspace reused), one after another
    ws = torch.empty(max(afmm.workspace_size(case, X.shape[0], "strict") for case, X, _ in host),
                     dtype=torch.uint8, device=dev)
    sp = stream.cuda_stream
    zs = [torch.empty_like(Z) for *_, Z in probs]

    def separate():
        for (case, Xd, Yd, _), Z2 in zip(probs, zs):
            f = afmm.afmm_multiply_caseA if case == "A" else afmm.afmm_multiply_caseB
            st = f(Xd.shape[0], Xd.data_ptr(), Yd.data_ptr(), Z2.data_ptr(), 0, ws.data_ptr(),
                   ws.numel(), sp)
            assert st == 0
    separate()
    torch.cuda.synchronize()
    sep_ms = event_time_ms(separate, max(1, min(args.steps, 5)), stream)
    same = all(torch.equal(a.view(torch.int32), b[3].view(torch.int32)) for a, b in zip(zs, probs))
    del zs, ws
    # spot parity: first row of a few products
    ok = True
    for t in (0, 1, len(host) // 2, len(host) - 1):
        case, X, Y = host[t]
        Zr, _ = oracle.strict_f32(case, X[:1], Y, rows=[0], x_rows_only=True)
        ok &= bool(np.array_equal(probs[t][3][:1].cpu().numpy().view(np.uint32), Zr.view(np.uint32)))
    frac = issued / (ms * 1e-3) / 1e12 / SINGLE_ISSUE_TADDS
    plan.close()
    log(f"bench: batched {ms:.3f} ms, {adds / (ms * 1e-3):.3e} adds/s, issued frac {frac:.3f}; "
        f"separate launches {sep_ms:.3f} ms")
    return {"workload": "512 products, n log-uniform [32,1024], d1,d2 ~ U(0.05,1), "
                        "integer U{0..R}, R in {3,15,63,255}, real U(-1,1)",
            "ms": ms, "useful_adds": adds, "useful_adds_per_s": adds / (ms * 1e-3),
            "separate_launches_ms": sep_ms,
            "separate_launches_useful_adds_per_s": adds / (sep_ms * 1e-3),
            # the same products, the same additions: useful adds/s of the one batched
            # launch over that of the products as separate calls
            "efficiency_vs_separate_launches": sep_ms / ms,
            "separate_launches_bit_identical": bool(same),
            # useful adds/s over that of the single n=4096 product
            "useful_rate_vs_single_launch": adds / (ms * 1e-3) / single_useful_per_s,
            "issued_lane_adds": issued,
            "issued_frac_of_single_issue_rate": frac,
            "issued_rate_vs_single_launch": frac / single_issued_frac,
            "bitexact_sampled_rows": ok,
            "timed": "whole plan launch (graph replay: prep, count, schedule, persistent kernel); "
                     "separate: 512 afmm_multiply_caseA/B calls in a row"}


def add_rate_probe(stream):
    """The device's binary32 add rate on straight-line v_add_f32 runs (the library's
    probe kernel, one block per compute unit) at 1, 2 and 4 waves per SIMD: the
    measured denominator beside the nominal one."""
    import ctypes

    import torch
    import paper_1308_2400_amd as afmm
    out = torch.empty(1024, dtype=torch.float32, device="cuda")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res = {}
    for wps in (1, 2, 4):
        adds = ctypes.c_uint64()

        def go():
            st = afmm.afmm_probe_add_rate(wps, 4000, out.data_ptr(), ctypes.byref(adds),
                                          stream.cuda_stream)
            assert st == 0
        for _ in range(20):  # settle the clock
            go()
        ms = event_time_ms(go, 10, stream)
        rate = adds.value / (ms * 1e-3)
        res[f"{wps}_waves_per_simd"] = {
            "adds_per_s": rate, "frac_of_nominal_peak": rate / 1e12 / PEAK_ADD_TFLOPS,
            "lane_adds_per_clk_per_cu_at_2.4GHz": rate / (cus * 2.4e9)}
    res["compute_units"] = cus
    res["kernel"] = "add_rate_probe_kernel: 16 accumulators x 8 adds per trip, 4000 trips"
    res["note"] = ("one wave issues at most one VALU instruction per 4 cycles; the doubled "
                   "binary32 rate needs two waves ready to issue on a SIMD")
    return res


# the paper's Table 1 (seconds, one Pentium at 1.6 GHz, single thread), for context:
# n -> (ijk, ikj, AFMM at mu' = 1, 3, 5, 7, 14, 21)
TABLE1_PAPER = {
    250: (0.411667, 0.328, 0.1752, 0.2784, 0.3316, 0.3498, 0.3188, 0.2874),
    500: (2.718667, 2.32, 0.918, 1.5406, 1.943, 2.331, 1.9122, 1.9874),
    750: (10.235, 7.75533, 2.8475, 4.9718, 6.38, 7.6826, 6.3218, 6.4328),
    1000: (25.125, 18.43233, 6.67175, 11.8064, 15.073, 18.2756, 14.9158, 15.3374),
    1250: (49.437, 35.75, 13.0897, 23.0705, 29.489, 35.594, 29.172, 29.9267),
    1500: (85.531, 61.688, 22.5625, 40.078, 50.9295, 61.718, 50.3515, 52.2),
    1750: (135.906, 98.515, 36.0235, 63.2655, 80.6235, 97.6955, 80.281, 81.9335),
    2000: (205.422, 147.078, 53.375, 94.6875, 120.8515, 145.8985, 119.516, 122.491),
}


def paper_seconds(n, mu):
    """The paper's Table 1 time for AFMM at (n, mu'), seconds."""
    return TABLE1_PAPER[n][2 + (1, 3, 5, 7, 14, 21).index(mu)]


def empirical_fit(rows):
    """Empirical order of the measured times (Section 2.2 bounds the work statistically by
    the expected number of additions): least-squares exponent b of time ~ n^b for each mu'
    and reading, and time = t0 + adds / rate over all sizes above the smallest (where the
    launch and the fixed passes dominate)."""
    import numpy as np
    fits = {}
    for mu in sorted({r["mu_prime"] for r in rows}):
        for yd in ("const", "uniform"):
            sel = [r for r in rows if r["mu_prime"] == mu and r["y_nonzeros"] == yd]
            if len(sel) < 3:
                continue
            ln_n = np.log([r["n"] for r in sel])
            b, _ = np.polyfit(ln_n, np.log([r["gpu_ms"] for r in sel]), 1)
            ba, _ = np.polyfit(ln_n, np.log([float(r["adds"]) for r in sel]), 1)
            fits[f"{mu}_{yd}"] = {"time_exponent_in_n": float(b), "adds_exponent_in_n": float(ba)}
    big = [r for r in rows if r["n"] > min(x["n"] for x in rows)]
    A = np.array([[1.0, float(r["adds"])] for r in big])
    t = np.array([r["gpu_ms"] for r in big])
    (t0, slope), *_ = np.linalg.lstsq(A, t, rcond=None)
    pred = A @ np.array([t0, slope])
    r2 = 1.0 - float(((t - pred) ** 2).sum() / ((t - t.mean()) ** 2).sum())
    return {"per_mu": fits,
            "time_vs_adds": {"t0_ms": float(t0), "adds_per_s": float(1e3 / slope), "r2": r2,
                             "rows": len(big)}}


# compacted-base configuration for a real factor with few non-zeros (autotuner's
# pick on the n=16384 case-A distribution at n = 2048..8192)
SPARSE_REAL_CONFIG = (4, 2, 16, 8, 1, 16)


def c5(args):
    """Case A, n=16384: X U(-1,1) with d1 = 0.05, Y Geometric(0.3) clipped to 0..255: the
    strict kernel beside the split form; strict rows bit-exact and the split's error
    against the binary64 product on sampled rows (64 rows i = 256 t + 17 plus the rows
    with the most and the fewest additions)."""
    import numpy as np
    import torch

    import gen
    import oracle
    import paper_1308_2400_amd as afmm
    stream = torch.cuda.current_stream()
    w = gen.caseA_n16384()
    n = w.n
    log("bench: generating caseA_n16384 (two 1 GiB matrices)")
    X, Y = w.X(), w.Y()
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    adds, rows = afmm.count_adds("A", Xd, Yd, rows=True)
    rows = rows.cpu().numpy()
    sample = sorted(set([256 * t + 17 for t in range(64)] + [int(rows.argmax()), int(rows.argmin())]))
    steps = max(1, min(args.steps, 3))
    Z = afmm.multiply("A", Xd, Yd)
    strict_ms = event_time_ms(lambda: afmm.multiply("A", Xd, Yd, out=Z), steps, stream)
    strict_launches = max(steps, 5)
    strict_median, strict_min = per_launch_ms(lambda: afmm.multiply("A", Xd, Yd, out=Z),
                                              strict_launches, stream)
    form = afmm.plain_form("A", Xd, Yd)
    log(f"bench: c5 strict plain call {strict_ms:.2f} ms (median {strict_median:.2f}, "
        f"min {strict_min:.2f}), form chosen on the device: mapping {form}")
    # the size-keyed form run explicitly (what the plain call ran before it chose
    # from the data)
    size_keyed = afmm.default_config("A", n)
    Zk = afmm.multiply("A", Xd, Yd, config=size_keyed)
    keyed_ms = event_time_ms(lambda: afmm.multiply("A", Xd, Yd, out=Zk, config=size_keyed),
                             steps, stream)
    log(f"bench: c5 strict size-keyed form {keyed_ms:.2f} ms")
    del Zk
    # the compacted-base form (lanes over each k's non-zero bases, Z block in LDS),
    # run explicitly
    Zc = afmm.multiply("A", Xd, Yd, config=SPARSE_REAL_CONFIG)
    acc_ms = event_time_ms(lambda: afmm.multiply("A", Xd, Yd, out=Zc, config=SPARSE_REAL_CONFIG),
                           steps, stream)
    log(f"bench: c5 strict compacted-base {acc_ms:.2f} ms")
    Zch = Zc.cpu().numpy()[sample]
    del Zc
    Zs = afmm.multiply("A", Xd, Yd, mode="split_bf16x3")
    split_ms = event_time_ms(lambda: afmm.multiply("A", Xd, Yd, mode="split_bf16x3", out=Zs),
                             steps, stream)
    log(f"bench: c5 split {split_ms:.2f} ms")
    Zh, Zsh = Z.cpu().numpy()[sample], Zs.cpu().numpy()[sample]
    Zr, _ = oracle.caseA_f32(X[sample], Y, rows=sample, x_rows_only=True)
    Z64 = oracle.product_f64("A", X[sample], Y, rows=sample, x_rows_only=True)
    out = {"metric": "case A n=16384 (C5): strict AFMM vs split-BF16x3", "unit": "ms",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic (seeded generator)",
           "dtype": "f32", "config": {"workload": w.name, "case": "A", "n": n, "d1": 0.05,
                                      "int_dist": "Geometric(0.3) clipped to [0,255]",
                                      "real_dist": "U(-1,1)"},
           "useful_adds": adds,
           "strict": {"ms": strict_ms, "ms_median": strict_median, "ms_min": strict_min,
                      "launches_timed_one_by_one": strict_launches,
                      "useful_adds_per_s": adds / (strict_ms * 1e-3),
                      "frac_of_add_peak": adds / (strict_ms * 1e-3) / 1e12 / PEAK_ADD_TFLOPS,
                      "bitexact_sampled_rows": bool(np.array_equal(Zh.view(np.uint32),
                                                                   Zr.view(np.uint32))),
                      "rel_frobenius_err_vs_f64": oracle.rel_frobenius(Zh, Z64),
                      "form_chosen_on_device": form,
                      "vs_best_explicit_form": strict_ms / min(keyed_ms, acc_ms)},
           "strict_size_keyed": {"ms": keyed_ms, "kernel_config": list(size_keyed),
                                 "frac_of_add_peak": adds / (keyed_ms * 1e-3) / 1e12
                                 / PEAK_ADD_TFLOPS},
           "strict_compacted_base": {
               "ms": acc_ms, "useful_adds_per_s": adds / (acc_ms * 1e-3),
               "frac_of_add_peak": adds / (acc_ms * 1e-3) / 1e12 / PEAK_ADD_TFLOPS,
               "bitexact_sampled_rows": bool(np.array_equal(Zch.view(np.uint32),
                                                            Zr.view(np.uint32))),
               "speedup_over_size_keyed": keyed_ms / acc_ms,
               "kernel_config": list(SPARSE_REAL_CONFIG)},
           "split": {"ms": split_ms, "effective_2n3_per_s": 2.0 * n ** 3 / (split_ms * 1e-3),
                     "mfma_frac_of_bf16_peak": 6.0 * n ** 3 / (split_ms * 1e-3) / 1e12
                     / PEAK_BF16_TFLOPS,
                     "rel_frobenius_err_vs_f64": oracle.rel_frobenius(Zsh, Z64),
                     "speedup_over_strict": strict_ms / split_ms},
           "err_sample": f"{len(sample)} rows"}
    print(json.dumps(out), flush=True)


def table1(args):
    """Section 2.3.1 / Table 1 grid: case A, d1 = 1/3, d2 = 1/2 for mu' <= 7 and 1/5, 2/5
    for 14 and 21.  The distribution of Y's non-zeros is not stated; both readings are run:
    every non-zero equal to mu', and Uniform{1..2mu'-1} (mean mu')."""
    import torch

    import gen
    import oracle
    import paper_1308_2400_amd as afmm
    stream = torch.cuda.current_stream()
    rows = []
    for n in gen.TABLE1_N:
        for mu in gen.TABLE1_MU:
            for ydist in ("const", "uniform"):
                w = gen.table1(n, mu, ydist)
                d1, d2 = w.real.density, w.int_.density
                X, Y = w.X(), w.Y()
                Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
                Z = afmm.multiply("A", Xd, Yd)
                adds = afmm.count_adds("A", Xd, Yd)
                ms = event_time_ms(lambda: afmm.multiply("A", Xd, Yd, out=Z), max(args.steps, 3),
                                   stream)
                r = {"n": n, "mu_prime": mu, "d1": d1, "d2": d2, "y_nonzeros": ydist,
                     "adds": adds, "expected_adds": w.expected_adds(), "gpu_ms": ms,
                     "adds_per_s": adds / (ms * 1e-3),
                     "paper_pentium_s": paper_seconds(n, mu)}
                if n == 250:  # the oracle (single thread) for the smallest size, bit for bit
                    t = time.perf_counter()
                    Zr, a2 = oracle.caseA_f32(X, Y)
                    r["cpu_oracle_s"] = time.perf_counter() - t
                    r["bitexact"] = bool((Z.cpu().numpy().view("u4") == Zr.view("u4")).all())
                    assert a2 == adds
                rows.append(r)
                log(f"table1 n={n} mu'={mu} {ydist}: {ms:.3f} ms, {adds:.3e} adds")
    out = {"metric": "Table 1 grid (case A): strict AFMM time per product", "unit": "ms",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic (seeded generator)",
           "paper_table1_seconds_pentium": {str(k): v for k, v in TABLE1_PAPER.items()},
           "empirical_fit": empirical_fit(rows), "rows": rows}
    print(json.dumps(out), flush=True)


# the form over the non-zeros of both factors (mapping 7): 16 waves, 2048-column bands
LOW_DENSITY_CONFIG = (7, 1, 32, 16, 1, 16)
LOW_DENSITY_N = (1024, 2048, 4096, 8192)


def low_density(args):
    """Section 2.2's low-density regime: d1 * d2 = 1/n (both densities n^-1/2), case A
    and case B, integer non-zeros U{1..7}, real ones U(-1,1).  The additions grow as n^2;
    the default strict form walks every k of every row block, the form over the
    non-zeros of both factors does work in proportion to the non-zero pairs.  Two rows
    per product checked bit for bit against the oracle; growth exponents fitted."""
    import numpy as np
    import torch

    import gen
    import oracle
    import paper_1308_2400_amd as afmm
    stream = torch.cuda.current_stream()
    rows = []
    for case in ("A", "B"):
        for n in LOW_DENSITY_N:
            d = 1.0 / math.sqrt(n)
            w = gen.Workload(f"lowdensity_{case}_n{n}", case, n, gen.RealSpec(gen.UNIFORMPM1, d),
                             gen.IntSpec(gen.INT_UNIFORM, d, 1, 7), gen.SEED0 + 7,
                             n + (1 if case == "B" else 0))
            X, Y = w.X(), w.Y()
            Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
            adds = afmm.count_adds(case, Xd, Yd)
            steps = max(args.steps, 3)
            # the plain call (it chooses its form on the device), the size-keyed
            # form and the row-list form, each called explicitly
            Zp = afmm.multiply(case, Xd, Yd)
            ms_plain = event_time_ms(lambda: afmm.multiply(case, Xd, Yd, out=Zp), steps, stream)
            keyed = afmm.default_config(case, n)
            Zd = afmm.multiply(case, Xd, Yd, config=keyed)
            ms_default = event_time_ms(lambda: afmm.multiply(case, Xd, Yd, out=Zd, config=keyed),
                                       steps, stream)
            Zl = afmm.multiply(case, Xd, Yd, config=LOW_DENSITY_CONFIG)
            ms_low = event_time_ms(
                lambda: afmm.multiply(case, Xd, Yd, out=Zl, config=LOW_DENSITY_CONFIG), steps,
                stream)
            sample = [n // 3, n - 1]
            Zr, _ = oracle.strict_f32(case, X[sample], Y, rows=sample, x_rows_only=True)
            ok = bool(np.array_equal(Zl.cpu().numpy()[sample].view(np.uint32), Zr.view(np.uint32))
                      and torch.equal(Zl.view(torch.int32), Zd.view(torch.int32))
                      and torch.equal(Zp.view(torch.int32), Zd.view(torch.int32)))
            form = afmm.plain_form(case, Xd, Yd)
            rows.append({"case": case, "n": n, "d1": d, "d2": d, "adds": adds,
                         "plain_ms": ms_plain, "plain_form": form,
                         "default_ms": ms_default, "default_config": list(keyed),
                         "low_density_ms": ms_low, "speedup": ms_default / ms_low,
                         "bitexact_sampled_rows": ok})
            log(f"lowdensity {case} n={n}: {adds:.3e} adds, plain call {ms_plain:.3f} ms "
                f"(mapping {form}), size-keyed form {ms_default:.3f} ms, "
                f"low-density form {ms_low:.3f} ms")
            del Xd, Yd, Zd, Zl, Zp
            torch.cuda.empty_cache()

    def exponent(case, key):
        sel = [r for r in rows if r["case"] == case]
        return float(np.polyfit(np.log([r["n"] for r in sel]), np.log([r[key] for r in sel]),
                                1)[0])
    fits = {case: {k: exponent(case, k) for k in ("adds", "plain_ms", "default_ms", "low_density_ms")}
            for case in ("A", "B")}
    out = {"metric": "low-density regime d1*d2 = 1/n: strict AFMM time per product", "unit": "ms",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic (seeded generator)",
           "low_density_config": list(LOW_DENSITY_CONFIG), "growth_exponents_in_n": fits,
           "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the product shards by rows with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    if args.lowdensity:
        return low_density(args)
    if args.table1:
        return table1(args)
    if args.c5:
        return c5(args)
    import numpy as np
    import torch

    import gen
    import paper_1308_2400_amd as afmm

    dev = torch.device("cuda:0")
    if args.copy_mb:
        src = torch.ones(args.copy_mb * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = gen.caseB_n4096(n=args.n)
    log(f"bench: generating {w.name}")
    X, Y = w.X(), w.Y()
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.from_numpy(Y).to(dev)
    n = w.n
    Z = torch.empty((n, n), dtype=torch.float32, device=dev)
    ws = torch.empty(afmm.workspace_size("B", n, "strict"), dtype=torch.uint8, device=dev)
    ws_split = torch.empty(afmm.workspace_size("B", n, "split"), dtype=torch.uint8, device=dev)
    total = torch.empty(1, dtype=torch.uint64, device=dev)
    flags = torch.empty(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    adds = afmm.count_adds("B", Xd, Yd)
    cfg = afmm.default_config("B", n)
    log(f"bench: counted adds {adds}, config {cfg}")

    def count():
        st = afmm.afmm_count_adds(1, n, Xd.data_ptr(), Yd.data_ptr(), total.data_ptr(), None,
                                  flags.data_ptr(), ws.data_ptr(), ws.numel(), sp)
        assert st == 0

    def strict():
        st = afmm.afmm_multiply_caseB(n, Xd.data_ptr(), Yd.data_ptr(), Z.data_ptr(), 0,
                                      ws.data_ptr(), ws.numel(), sp)
        assert st == 0

    def step():
        count()
        strict()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    step_ms = event_time_ms(step, args.steps, stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    strict_ms = event_time_ms(strict, args.steps, stream)
    strict_launches = max(args.steps, 20)
    strict_median, strict_min = per_launch_ms(strict, strict_launches, stream)
    count_ms = event_time_ms(count, args.steps, stream)
    log(f"bench: step {step_ms:.3f} ms (wall {wall_ms:.3f}), strict {strict_ms:.3f} ms, "
        f"count {count_ms:.3f} ms")

    # parity spot check of the timed result (sampled rows, bit for bit)
    import oracle
    rows = [0, 1, n // 3, n - 1]
    Zr, _ = oracle.strict_f32("B", X[rows], Y, rows=rows, x_rows_only=True)
    bitexact = bool(np.array_equal(Z.cpu().numpy()[rows].view(np.uint32), Zr.view(np.uint32)))
    assert total.cpu().view(torch.int64).item() == adds

    useful_per_s = adds / (step_ms * 1e-3)
    strict_tflops = adds / (strict_ms * 1e-3) / 1e12
    eff_2n3 = 2.0 * n ** 3 / (strict_ms * 1e-3)
    issued = int(X.astype(np.int64).sum()) * n  # lane-slot adds the count-uniform mapping issues

    out = {
        "metric": "n=4096 useful adds/s + effective 2n^3/s: strict AFMM vs split-BF16 MFMA at 1e-6 rel",
        "value": useful_per_s,
        "unit": "useful adds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": w.name, "case": "B", "n": n, "d1": 0.3, "d2": 0.9,
                   "int_dist": "Poisson(3) clipped to [0,255]", "real_dist": "N(0,1)",
                   "kernel_config": list(cfg), "form_chosen_on_device": afmm.plain_form("B", Xd, Yd)},
        "useful_adds": adds,
        "strict": {"ms": strict_ms, "ms_median": strict_median, "ms_min": strict_min,
                   "launches_timed_one_by_one": strict_launches,
                   "useful_adds_per_s": adds / (strict_ms * 1e-3),
                   "effective_2n3_per_s": eff_2n3, "issued_lane_adds": issued,
                   "issued_frac_of_single_issue_rate": issued / (strict_ms * 1e-3) / 1e12 / SINGLE_ISSUE_TADDS,
                   "bitexact_sampled_rows": bitexact},
        "count_ms": count_ms,
        "roofline": {"bound": "alu", "achieved": strict_tflops, "peak": PEAK_ADD_TFLOPS,
                     "unit": "TFLOP/s", "frac": strict_tflops / PEAK_ADD_TFLOPS,
                     "traffic": measured_traffic(cfg),
                     "kernel": {0: "rep_uniform_kernel", 2: "rep_direct_kernel",
                                3: "rep_sparse_kernel"}.get(cfg[0], "strict kernel")
                               + " (strict, one launch = one n=4096 product)"},
    }

    out["add_peak_probe"] = add_rate_probe(stream)
    log("bench: add-rate probe " + ", ".join(
        f"{k} {v['frac_of_nominal_peak']:.3f}" for k, v in out["add_peak_probe"].items()
        if isinstance(v, dict)))

    if not args.no_split:
        Zs = torch.empty_like(Z)

        def split():
            st = afmm.afmm_multiply_caseB(n, Xd.data_ptr(), Yd.data_ptr(), Zs.data_ptr(), 1,
                                          ws_split.data_ptr(), ws_split.numel(), sp)
            assert st == 0

        for _ in range(args.warmup):
            split()
        split_ms = event_time_ms(split, args.steps, stream)
        rows = list(range(0, n, n // 32))
        Z64 = oracle.product_f64("B", X[rows], Y, rows=rows, x_rows_only=True)
        err = oracle.rel_frobenius(Zs.cpu().numpy()[rows], Z64)
        err_strict = oracle.rel_frobenius(Z.cpu().numpy()[rows], Z64)
        out["split"] = {"ms": split_ms, "effective_2n3_per_s": 2.0 * n ** 3 / (split_ms * 1e-3),
                        "mfma_tflops": 6.0 * n ** 3 / (split_ms * 1e-3) / 1e12,
                        "mfma_frac_of_bf16_peak": 6.0 * n ** 3 / (split_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS,
                        "rel_frobenius_err_vs_f64": err, "err_sample": f"{len(rows)} rows",
                        "strict_rel_frobenius_err_vs_f64": err_strict,
                        "speedup_over_strict": strict_ms / split_ms}
        log(f"bench: split {split_ms:.3f} ms err {err:.2e}")

    if not args.no_batched:
        out["batched"] = bench_batched(args, stream, out["strict"]["issued_frac_of_single_issue_rate"],
                                       out["strict"]["useful_adds_per_s"])

    if not args.no_cpu_baseline:
        log("bench: cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w, X, Y, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
