#!/usr/bin/env python3
"""Benchmark: all-pairs binary mutual information on one MI355X.

One step = one full pass of the hot path (mi_all_pairs_ex through the C ABI
with the library's choices: at this shape the byte matrix is converted to FP4
(E2M1) codes, then the fused kernel runs the Gram on the FP4 matrix cores,
with the column sums, the MI epilogue and the tile and mirror write-back)
over the 1,000,000 x 4,096 synthetic fingerprint-like matrix, already
resident in HBM.  --gram int8 runs the int8 Gram on the bytes instead.

Prints one JSON line:
  value      pair-updates/s = m * n (n + 1) / 2 per step / seconds per step
             (conversion pass included)
  roofline   the fused kernel (the dominant one) against the matrix-core peak
             of its operand type (2 ops per pair-update per row), timed alone
             with HIP events on its stream
  cpu_baseline  the CPU oracle on a bounded column sample of the same matrix
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT8_OPS = 5.0e15      # MI355X dense int8 matrix-core peak, ops/s
PEAK_FP4_OPS = 10.1e15      # MI355X dense FP4 (E2M1) matrix-core peak, ops/s
GRAM_NAMES = {1: "int8", 2: "fp4"}
PEAK_HBM = 8.0e12           # bytes/s

WORKLOADS = {
    "large_1000000x4096": "spec_large",
    "mid_100000x1024": "spec_mid",
    "small_1000x200": "spec_small",
    "outbound_2000x8192": "spec_outbound",
}
OUTPUT_BOUND_ROWS = 2500    # below this m the n^2 FP32 write-back outweighs the Gram (roofline crossover)


KERNEL_SOURCES = ("mi_device.hpp", "mi_internal.hpp", "mi_kernels.hip")


def kernel_source_hash() -> str:
    """Hash of the device-code sources (the kernels and their launch shapes)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_19702_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def plain_kernel_name(tile: int, gram: int) -> str:
    """Demangled name of the fused kernel for a tile id and Gram (input layout 0: bytes, 2: FP4)."""
    return "mi::k_plain<mi::Cfg<%d, 2, %d, 4>, %d>" % (((128, 2) if tile == 1 else (256, 4)) + (2 if gram == 2 else 0,))


def load_traffic(workload: str, tile: int, splits: int, kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources for the same kernel, tile and
    split count."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_source_hash():
        return None
    if rec.get("tile") != tile or rec.get("splits") != splits or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(spec, target_s: float):
    """The oracle (all pairs of a column subset, every row) on the host cores."""
    import numpy as np
    import oracle
    from paper_2411_19702_amd import synth
    rng = np.random.default_rng(5)
    m = spec.m

    def run(ncols):
        cols = sorted(int(c) for c in rng.choice(spec.n, size=ncols, replace=False))
        Xs = synth.columns(spec, cols).numpy()
        t0 = time.perf_counter()
        oracle.all_pairs(Xs)
        return time.perf_counter() - t0, ncols, Xs

    dt, k, _ = run(6)
    # pairs scale as k(k+1)/2: pick k for about target_s seconds
    per_pair = dt / (k * (k + 1) / 2)
    k2 = int(max(6, min(spec.n, (2 * target_s / max(per_pair, 1e-9)) ** 0.5)))
    dt, k, Xs = run(k2)
    pu = m * k * (k + 1) / 2
    # One thread: pairs of the same sampled matrix, one call at a time (each
    # call's parallel loop has a single iteration), about 2 s of them; only
    # where a pair's rows outweigh the per-call overhead.
    single = None
    if m >= 100_000:
        t0 = time.perf_counter()
        oracle.pairs(Xs, [0], [1])
        per = max(time.perf_counter() - t0, 1e-6)
        npairs = int(max(4, min(k * (k + 1) // 2, 2.0 / per)))
        ij = [(int(a), int(b)) for a, b in zip(rng.integers(0, k, size=npairs), rng.integers(0, k, size=npairs))]
        t0 = time.perf_counter()
        for a, b in ij:
            oracle.pairs(Xs, [min(a, b)], [max(a, b)])
        dt1 = time.perf_counter() - t0
        single = (len(ij) * m / dt1, f"{len(ij)} random pairs of the same {k}-column sample, one call each; {dt1:.2f} s")
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": pu / dt,
        "unit": "pair-updates/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"all {k * (k + 1) // 2} pairs (i <= j) of {k} random columns x all {m} rows of the same matrix; {dt:.2f} s",
        "single_thread_value": single[0] if single else None,
        "single_thread_sample": single[1] if single else None,
        "cpu_model": model,
        "nproc": os.cpu_count(),
    }


def roofline(m: int, in_bytes: int, n: int, kernel_s: float, ops_per_s: float, traffic, tile: int, gram: int) -> dict:
    """Roofline object for the fused kernel: against the matrix-core peak of its
    operand type (int8 or FP4), or, for output-bound shapes (m below the
    crossover), against HBM with the algorithmic bytes (the kernel's input read
    once + the n x n FP32 output)."""
    kern = plain_kernel_name(tile, gram)
    if m < OUTPUT_BOUND_ROWS:
        gbs = (in_bytes + 4 * n * n) / kernel_s
        return {"bound": "hbm", "achieved": gbs / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": gbs / PEAK_HBM, "traffic": traffic, "kernel": kern, "kernel_ms": kernel_s * 1e3}
    peak = PEAK_FP4_OPS if gram == 2 else PEAK_INT8_OPS
    return {"bound": "mfma", "achieved": ops_per_s / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": ops_per_s / peak, "traffic": traffic, "kernel": kern, "kernel_ms": kernel_s * 1e3}


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def bench_plain(dev, workload: str, steps: int = 30, tune: bool = False):
    """One named single-dataset workload through mi_all_pairs_ex: median kernel
    time (HIP events on the launch stream), blocking-call latency, pair-updates/s,
    fraction of the int8 peak and algorithmic HBM rate (X once + FP32 output)."""
    import torch
    from paper_2411_19702_amd import mi, synth
    spec = getattr(synth, WORKLOADS[workload])()
    X = synth.generate(spec, device=dev)
    m, n = spec.m, spec.n
    out = torch.empty((n, n), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    tuned = None
    if tune:
        tile, splits, best = mi.mi_tune(m, n, X.stride(0))
        tuned = {"tile": [None, 128, 256][tile], "splits": splits}
    tile, splits, gram = mi.mi_plan_ex(X)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        mi.mi_all_pairs_ex(X, out=out, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(stream)
        mi.mi_all_pairs_ex(X, out=out, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ks = sorted(e0.elapsed_time(e1) / 1e3 for e0, e1 in ev)
    k = ks[len(ks) // 2]
    lat = []
    for _ in range(steps):
        t0 = time.perf_counter()
        mi.mi_all_pairs_ex(X, out=out, stream=stream)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    pu = m * n * (n + 1) / 2
    nbytes = m * X.stride(0) + 4 * n * n
    del X, out
    torch.cuda.empty_cache()
    peak = PEAK_FP4_OPS if gram == 2 else PEAK_INT8_OPS
    return {"workload": workload, "m": m, "n": n, "tile": [None, 128, 256][tile], "splits": splits,
            "gram": GRAM_NAMES[gram], "tuned": tuned, "call_ms_median_on_stream": k * 1e3,
            "call_latency_ms_median": _pct(lat, 50) * 1e3, "pair_updates_per_s": pu / k,
            "frac_int8_peak": 2 * pu / k / PEAK_INT8_OPS, "frac_gram_dtype_peak": 2 * pu / k / peak,
            "hbm_algorithmic_GBps": nbytes / k / 1e9, "frac_hbm_peak": nbytes / k / PEAK_HBM}


def bench_sparse(dev, thr: float = 0.01, reps: int = 3):
    """Sparse threshold output on the wide 20,000 x 32,768 workload: only the
    pairs with MI >= thr are written, against the dense 4.3 GB matrix."""
    import torch
    from paper_2411_19702_amd import mi, synth
    spec = synth.spec_wide()
    X = synth.generate(spec, device=dev)
    m, n = spec.m, spec.n
    cap = 4 * n
    pairs = torch.empty((cap, 3), dtype=torch.int32, device=dev)
    count = torch.empty((1,), dtype=torch.int64, device=dev)
    prob_sparse = mi.make_problem(X, None, pairs=pairs, pairs_count=count, pairs_threshold=thr)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    import ctypes
    t_sparse = timed(lambda: mi._check(mi.lib().mi_all_pairs_ex(ctypes.byref(prob_sparse), mi._stream_handle(stream))))
    found = int(count.item())
    out = torch.empty((n, n), dtype=torch.float32, device=dev)
    t_dense = timed(lambda: mi.mi_all_pairs_ex(X, out=out, stream=stream))
    dense_count = int(torch.triu(out >= thr, diagonal=1).sum().item())
    del out
    torch.cuda.empty_cache()
    pu = m * n * (n + 1) / 2
    return {"workload": f"wide_{m}x{n}", "threshold_bits": thr, "pairs_found": found,
            "pairs_in_dense_filter": dense_count, "sparse_ms": t_sparse * 1e3, "dense_ms": t_dense * 1e3,
            "sparse_pair_updates_per_s": pu / t_sparse, "dense_output_bytes": 4 * n * n,
            "sparse_output_bytes": 12 * min(found, cap)}


def bench_sparse_input(dev, densities=(0.001, 0.005, 0.02), reps: int = 3):
    """The sparse-input path against the dense int8 path on 1,000,000 x 4,096
    matrices of mean density d (p_j ~ U[0, 2d]): blocking call time each."""
    import torch
    from paper_2411_19702_amd import mi, synth
    res = []
    for d in densities:
        spec = synth.spec_random(11, 1_000_000, 4096, 0.0, 2.0 * d)
        X = synth.generate(spec, device=dev)
        out = torch.empty((4096, 4096), dtype=torch.float32, device=dev)
        row = {"density": d}
        for name, algo in (("dense", mi.MI_ALGO_DENSE), ("sparse", mi.MI_ALGO_SPARSE), ("auto", mi.MI_ALGO_AUTO)):
            mi.mi_all_pairs_ex(X, out=out, algo=algo)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                mi.mi_all_pairs_ex(X, out=out, algo=algo)
                torch.cuda.synchronize()
            row[name + "_ms"] = (time.perf_counter() - t0) / reps * 1e3
        res.append(row)
        print(f"[sparse-input] {row}", file=sys.stderr, flush=True)
        del X, out
        torch.cuda.empty_cache()
    return {"workload": "1000000x4096, p_j ~ U[0, 2d]", "rows": res}


def bench_categorical(dev, reps: int = 5):
    """Categorical (genotype-like, 3 codes per column) all-pairs MI: blocking
    call time, which covers the indicator expansion, the counts-only Gram of
    the N = 2 v indicator columns and the per-pair contingency reduce."""
    import torch
    from paper_2411_19702_amd import mi, synth
    res = []
    for m, v in ((1_000_000, 2048), (100_000, 8192)):
        spec = synth.spec_genotypes(m=m, v=v)
        X = synth.cat_generate(spec, device=dev)
        levels = [int(x) for x in spec.levels]
        out = torch.empty((v, v), dtype=torch.float32, device=dev)
        # The indicator Gram's matrix instructions: the library's choice for an m x N byte
        # problem (mi_plan_ex reads only the shape of its placeholder).
        probe = torch.empty((m, mi.mi_cat_indicators(levels)), dtype=torch.uint8, device=dev)
        gram = mi.mi_plan_ex(probe)[2]
        del probe
        mi.mi_all_pairs_categorical(X, levels, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            mi.mi_all_pairs_categorical(X, levels, out=out)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        N = mi.mi_cat_indicators(levels)
        row = {"workload": f"genotypes_{m}x{v}", "levels": 3, "indicator_columns": N, "ms": t * 1e3,
               "variable_pairs_per_s": v * (v + 1) / 2 / t,
               "gram": GRAM_NAMES[gram], "gram_ops_per_s": 2.0 * m * N * (N + 1) / 2 / t}
        res.append(row)
        print(f"[categorical] {row}", file=sys.stderr, flush=True)
        del X, out
        torch.cuda.empty_cache()
    return res


def bench_packed(dev, reps: int = 10):
    """Packed inputs on the 1,000,000 x 4,096 workload: the int8 byte kernel;
    bit-packed input (8x fewer input bytes) on the int8 Gram and on the FP4
    Gram (the library's choice), and its packing pass; FP4 input (2x fewer
    bytes, FP4 Gram) and its packing pass; the byte call with the FP4 Gram
    (conversion included).  Timed with HIP events on the stream."""
    import torch
    from paper_2411_19702_amd import mi, synth
    spec = synth.spec_large()
    X = synth.generate(spec, device=dev)
    n = spec.n
    out = torch.empty((n, n), dtype=torch.float32, device=dev)
    P = mi.mi_pack_bits(X)
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    Q = mi.mi_pack_fp4(X)
    t_bytes = timed(lambda: mi.mi_all_pairs_ex(X, out=out, gram=mi.MI_GRAM_INT8))
    t_packed = timed(lambda: mi.mi_all_pairs_ex(P, out=out, n=n, packed=True, gram=mi.MI_GRAM_INT8))
    t_packed4 = timed(lambda: mi.mi_all_pairs_ex(P, out=out, n=n, packed=True))
    t_pack = timed(lambda: mi.mi_pack_bits(X, out=P))
    t_fp4 = timed(lambda: mi.mi_all_pairs_ex(Q, out=out, n=n, packed=mi.MI_INPUT_FP4))
    t_pack4 = timed(lambda: mi.mi_pack_fp4(X, out=Q))
    t_bytes_fp4 = timed(lambda: mi.mi_all_pairs_ex(X, out=out, gram=mi.MI_GRAM_FP4))
    pu = spec.m * n * (n + 1) / 2
    row = {"workload": f"large_{spec.m}x{n}", "bytes_ms": t_bytes, "packed_ms": t_packed, "pack_pass_ms": t_pack,
           "pack_then_packed_ms": t_pack + t_packed, "input_bytes": spec.m * n, "packed_input_bytes": P.numel(),
           "packed_pair_updates_per_s": pu / (t_packed * 1e-3),
           "packed_int8_frac": 2 * pu / (t_packed * 1e-3) / PEAK_INT8_OPS,
           "packed_fp4_gram_ms": t_packed4, "packed_fp4_gram_pair_updates_per_s": pu / (t_packed4 * 1e-3),
           "packed_fp4_gram_frac": 2 * pu / (t_packed4 * 1e-3) / PEAK_FP4_OPS,
           "fp4_input_ms": t_fp4, "fp4_pack_pass_ms": t_pack4, "fp4_input_bytes": Q.numel(),
           "bytes_fp4_gram_ms": t_bytes_fp4, "fp4_pair_updates_per_s": pu / (t_fp4 * 1e-3),
           "fp4_frac": 2 * pu / (t_fp4 * 1e-3) / PEAK_FP4_OPS}
    print(f"[packed] {row}", file=sys.stderr, flush=True)
    del X, P, Q, out
    torch.cuda.empty_cache()
    return row


def bench_library_gemm(dev, reps: int = 10):
    """Context, not the product: the vendor int8 GEMM (torch._int_mm, which
    calls hipBLASLt on ROCm) computing the full square X^T X of the same
    matrix, beside this library's call that computes only i <= j and also
    produces the column sums and MI.  Both are timed with HIP events on the
    current stream; the library GEMM's operands are contiguous (X^T is
    materialised once, outside the timed region)."""
    import torch
    from paper_2411_19702_amd import mi, synth
    res = []
    for spec in (synth.spec_mid(), synth.spec_large()):
        X = synth.generate(spec, device=dev)
        m, n = spec.m, spec.n
        assert X.shape == (m, n) and X.is_contiguous()
        A = X.view(torch.int8).t().contiguous()
        B = X.view(torch.int8)
        out = torch.empty((n, n), dtype=torch.float32, device=dev)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        t_lib = timed(lambda: torch._int_mm(A, B))
        t_mi8 = timed(lambda: mi.mi_all_pairs_ex(X, out=out, gram=mi.MI_GRAM_INT8))
        t_mi = timed(lambda: mi.mi_all_pairs_ex(X, out=out))
        full_ops = 2.0 * m * n * n
        tri_ops = 2.0 * m * n * (n + 1) / 2
        row = {"workload": f"{spec.name}", "library_gemm_ms": t_lib,
               "library_gemm_full_square_ops_per_s": full_ops / (t_lib * 1e-3),
               "library_gemm_int8_frac": full_ops / (t_lib * 1e-3) / 5.0e15,
               "mi_all_pairs_int8_gram_ms": t_mi8, "mi_all_pairs_int8_gram_frac": tri_ops / (t_mi8 * 1e-3) / 5.0e15,
               "mi_all_pairs_ms": t_mi, "mi_all_pairs_gram": GRAM_NAMES[mi.mi_plan_ex(X)[2]],
               "speedup_vs_library_gemm": t_lib / t_mi}
        print(f"[library_gemm] {row}", file=sys.stderr, flush=True)
        res.append(row)
        del X, A, B, out
        torch.cuda.empty_cache()
    return res


def bench_batched(dev, reps: int = 10):
    """256 independent datasets: one persistent launch vs a replayed hipGraph
    of plain launches vs 256 sequential plain calls (same results, bitwise)."""
    import torch
    from paper_2411_19702_amd import mi, synth
    specs = synth.specs_batched()
    Xs = [synth.generate(s, device=dev) for s in specs]
    outs = [torch.empty((s.n, s.n), dtype=torch.float32, device=dev) for s in specs]
    # The batch as one C array of problems, built once (as a C caller would).
    probs = mi.problem_array([mi.make_problem(X, o) for X, o in zip(Xs, outs)])
    pu = sum(s.m * s.n * (s.n + 1) / 2 for s in specs)
    res = {"workload": "batched_256 (m log-uniform [500, 50000], n U[64, 2048])", "datasets": len(specs),
           "pair_updates": pu}
    for name, mode in (("persistent", mi.MI_BATCH_PERSISTENT), ("graph", mi.MI_BATCH_GRAPH),
                       ("sequential", mi.MI_BATCH_SEQUENTIAL)):
        mi.mi_all_pairs_batched(probs, mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            mi.mi_all_pairs_batched(probs, mode=mode)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[name] = {"ms": dt * 1e3, "pair_updates_per_s": pu / dt}
    # The batch autotuner on the same batch: its pick, then the persistent
    # mode timed again under the tuned plan (heuristic timed above).
    t0 = time.perf_counter()
    tuned_ms, heur_ms = mi.mi_tune_batched(probs)
    tune_s = time.perf_counter() - t0
    tiles, splits = mi.mi_plan_batched(probs)
    mi.mi_all_pairs_batched(probs, mode=mi.MI_BATCH_PERSISTENT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mi.mi_all_pairs_batched(probs, mode=mi.MI_BATCH_PERSISTENT)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    res["persistent_tuned"] = {"ms": dt * 1e3, "pair_updates_per_s": pu / dt, "tuner_ms": tuned_ms,
                               "tuner_heuristic_ms": heur_ms, "tuning_s": tune_s,
                               "tiles_256": tiles.count(mi.MI_TILE_256), "tiles_128": tiles.count(mi.MI_TILE_128),
                               "units_splits_total": int(sum(splits))}
    mi.mi_tuner_clear()
    del Xs, outs
    torch.cuda.empty_cache()
    return res


def bench_served(dev, count: int = 300, loads=(0.5, 0.8, 0.95, 1.5), slots: int = 3):
    """Poisson arrivals of MI requests (m log-uniform [1k, 200k], n log-uniform
    [128, 8192], densities U[0.005, 0.5]): the continuous-batching server vs
    one-at-a-time plain solves, both replayed at lambda = load * mu for each
    load, mu = the plain one-at-a-time capacity.  Latency runs from the
    scheduled arrival to result-ready; both paths are warmed first."""
    import torch
    from paper_2411_19702_amd import mi, synth
    trace = synth.request_trace(count=count, qps=1.0)
    specs = [r.spec for r in trace]
    Xs = [synth.generate(s, device=dev) for s in specs]
    outs = [torch.empty((s.n, s.n), dtype=torch.float32, device=dev) for s in specs]
    torch.cuda.synchronize()
    pu = sum(s.m * s.n * (s.n + 1) / 2 for s in specs)
    budget = 200 << 30
    # capacity of plain one-at-a-time solves (warm)
    for X, o in zip(Xs, outs):
        mi.mi_all_pairs_ex(X, out=o)
    torch.cuda.synchronize()
    svc = []
    for X, o in zip(Xs, outs):
        t0 = time.perf_counter()
        mi.mi_all_pairs_ex(X, out=o)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t0)
    mu = 1.0 / (sum(svc) / len(svc))

    def wait_until(t_abs):
        while True:
            d = t_abs - time.perf_counter()
            if d <= 0:
                return
            time.sleep(min(d, 2e-4) if d > 3e-4 else 0)

    res = {"workload": f"served: {count} Poisson requests, m log-uniform [1000, 200000], "
                       f"n log-uniform [128, 8192], densities U[0.005, 0.5]",
           "mu_req_per_s": mu, "budget_bytes": budget, "server_slots": slots, "loads": []}
    with mi.Server(hbm_budget_bytes=budget, max_slots=slots) as srv:
        for t in [srv.submit(X, o) for X, o in zip(Xs, outs)]:      # warm the server's streams
            srv.wait(t, timeout_s=300)
        for load in loads:
            lam = load * mu
            arrivals = [r.arrival_s / lam for r in trace]     # the unit-rate Poisson trace scaled to lambda
            # one at a time, first come first served
            t_start = time.perf_counter()
            lat_plain = []
            for a, X, o in zip(arrivals, Xs, outs):
                wait_until(t_start + a)
                mi.mi_all_pairs_ex(X, out=o)
                torch.cuda.synchronize()
                lat_plain.append(time.perf_counter() - (t_start + a))
            span_plain = time.perf_counter() - t_start
            # continuous batching
            st0 = srv.stats()
            t_start = time.perf_counter()
            tickets, late = [], []
            for a, X, o in zip(arrivals, Xs, outs):
                wait_until(t_start + a)
                late.append(time.perf_counter() - (t_start + a))
                tickets.append(srv.submit(X, o))
            lat_srv = [lt + srv.wait(t, timeout_s=300) for lt, t in zip(late, tickets)]
            span_srv = time.perf_counter() - t_start
            st = srv.stats()
            res["loads"].append({
                "load": load, "lambda_req_per_s": lam,
                "server": {"p50_ms": _pct(lat_srv, 50) * 1e3, "p99_ms": _pct(lat_srv, 99) * 1e3,
                           "pair_updates_per_s": pu / span_srv, "batches": st["batches"] - st0["batches"],
                           "max_in_flight": st["max_in_flight"]},
                "one_at_a_time": {"p50_ms": _pct(lat_plain, 50) * 1e3, "p99_ms": _pct(lat_plain, 99) * 1e3,
                                  "pair_updates_per_s": pu / span_plain},
            })
            print(f"[served] load {load}: server p50 {res['loads'][-1]['server']['p50_ms']:.2f} ms "
                  f"p99 {res['loads'][-1]['server']['p99_ms']:.2f} ms; one-at-a-time "
                  f"p50 {res['loads'][-1]['one_at_a_time']['p50_ms']:.2f} ms "
                  f"p99 {res['loads'][-1]['one_at_a_time']['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    del Xs, outs
    torch.cuda.empty_cache()
    return res


def run_extras(dev, extras, args) -> dict:
    rec = {}
    if "configs" in extras:
        rec["configs"] = [bench_plain(dev, "small_1000x200"), bench_plain(dev, "mid_100000x1024"),
                          bench_plain(dev, "mid_100000x1024", tune=True), bench_plain(dev, "outbound_2000x8192"),
                          bench_plain(dev, "outbound_2000x8192", tune=True)]
    if "batched" in extras:
        rec["batched"] = bench_batched(dev)
    if "served" in extras:
        rec["served"] = bench_served(dev, slots=args.served_slots)
    if "sparse" in extras:
        rec["sparse"] = bench_sparse(dev)
    if "sparse_input" in extras:
        rec["sparse_input"] = bench_sparse_input(dev)
    if "categorical" in extras:
        rec["categorical"] = bench_categorical(dev)
    if "packed" in extras:
        rec["packed"] = bench_packed(dev)
    if "library_gemm" in extras:
        rec["library_gemm"] = bench_library_gemm(dev)
    return rec


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_1000000x4096", choices=sorted(WORKLOADS))
    ap.add_argument("--epilogue", type=int, default=0, help="0 fp32, 1 fp32 + fp64 fallback, 2 fp64")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target oracle time for cpu_baseline (0: skip)")
    ap.add_argument("--tune", action="store_true", help="run the autotuner for this shape first")
    ap.add_argument("--pitch", type=int, default=0, help="row pitch of X in bytes (0: dense, pitch = n)")
    ap.add_argument("--shape", default="", help="M,N: time a random M x N matrix instead of a named workload")
    ap.add_argument("--tile", type=int, default=0, help="force a tile config (1: 128, 2: 256)")
    ap.add_argument("--splits", type=int, default=0, help="force the K-split count")
    ap.add_argument("--gram", default="auto", choices=("auto", "int8", "fp4"),
                    help="matrix instructions of the Gram (auto: the library's choice)")
    ap.add_argument("--no-extras", action="store_true", help="skip the extra measurements")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the extra measurements named by --extras (no headline line)")
    ap.add_argument("--extras", default="configs,batched,served,sparse,sparse_input,categorical,packed,library_gemm",
                    help="comma list of extra measurements: configs (the 1000 x 200 and 100000 x 1024 "
                         "workloads), batched (256 datasets), served (Poisson request trace), sparse (threshold "
                         "output on 20000 x 32768), sparse_input (sparse-input path at 1000000 x 4096), "
                         "categorical (genotype-like 3-code data), packed (bit-packed input), library_gemm (the "
                         "vendor int8 GEMM of the full square X^T X, for context)")
    ap.add_argument("--served-slots", type=int, default=3, help="server slots (streams) in the served measurement")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run a plain device copy of MIB MiB per step "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (got --gpus {args.gpus}); "
              "the path would shard by output tiles or by rows, which is not built here", file=sys.stderr)
        return 2

    import torch
    from paper_2411_19702_amd import mi, synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            torch.add(src, 0, out=dst)  # one elementwise kernel: reads nbytes, writes nbytes
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": args.warmup + args.steps}), flush=True)
        return 0
    if args.extras_only:
        print(json.dumps({"extras": run_extras(dev, set(args.extras.split(",")), args)}), flush=True)
        return 0
    if args.shape:
        sm, sn = (int(v) for v in args.shape.split(","))
        spec = synth.spec_random(7, sm, sn, 0.001, 0.2)
        args.workload = f"random_{sm}x{sn}"
    else:
        spec = getattr(synth, WORKLOADS[args.workload])()
    if args.pitch:
        spec.ldx = args.pitch
    m, n = spec.m, spec.n
    X = synth.generate(spec, device=dev)[:, :n]
    out = torch.empty((n, n), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    if args.tune:
        mi.mi_tune(m, n, n)
    gram_req = {"auto": mi.MI_GRAM_AUTO, "int8": mi.MI_GRAM_INT8, "fp4": mi.MI_GRAM_FP4}[args.gram]
    kw = dict(epilogue=args.epilogue, tile=args.tile, splits=args.splits, gram=gram_req)
    tile, splits, gram = mi.mi_plan_ex(X, **kw)
    stream = torch.cuda.current_stream()

    def step():
        mi.mi_all_pairs_ex(X, out=out, stream=stream, **kw)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    avg_step_s = sum(step_ms) / len(step_ms) / 1e3
    # The dominant kernel alone: with the FP4 Gram a step is the conversion
    # pass plus the fused kernel, so each is timed by itself, the fused kernel
    # on the converted input (same kernel, plan and stream).
    conversion = None
    avg_kernel_s, in_bytes = avg_step_s, m * X.stride(0)

    def timed(fn):
        fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for e0, e1 in evs:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return sum(e0.elapsed_time(e1) for e0, e1 in evs) / len(evs) / 1e3

    if gram == mi.MI_GRAM_FP4:
        Q = mi.mi_pack_fp4(X)
        kq = dict(kw, gram=mi.MI_GRAM_AUTO)
        avg_kernel_s = timed(lambda: mi.mi_all_pairs_ex(Q, out=out, n=n, packed=mi.MI_INPUT_FP4, stream=stream, **kq))
        conv_s = timed(lambda: mi.mi_pack_fp4(X, out=Q, stream=stream))
        in_bytes = Q.numel()
        conversion = {"kernel": "mi::k_pack_fp4", "ms": conv_s * 1e3, "bytes": m * X.stride(0) + Q.numel(),
                      "GBps": (m * X.stride(0) + Q.numel()) / conv_s / 1e9}
        del Q

    pu_per_step = m * n * (n + 1) / 2
    value = pu_per_step * args.steps / wall
    achieved = 2.0 * pu_per_step / avg_kernel_s
    # The fused kernel on the int8 Gram (int8 x int8 -> int32 matrix instructions on the
    # bytes), timed the same way on the same matrix: its fraction of the int8 peak.
    int8_kernel = None
    if gram == mi.MI_GRAM_FP4 and m >= OUTPUT_BOUND_ROWS:
        k8 = dict(kw, gram=mi.MI_GRAM_INT8)
        tile8, splits8, _ = mi.mi_plan_ex(X, **k8)
        t8 = timed(lambda: mi.mi_all_pairs_ex(X, out=out, stream=stream, **k8))
        int8_kernel = {"kernel": plain_kernel_name(tile8, mi.MI_GRAM_INT8), "tile": [None, 128, 256][tile8],
                       "splits": splits8, "ms": t8 * 1e3, "achieved_TOPS": 2.0 * pu_per_step / t8 / 1e12,
                       "frac_int8_peak": 2.0 * pu_per_step / t8 / PEAK_INT8_OPS}
    traffic = load_traffic(args.workload, [None, 128, 256][tile], splits, plain_kernel_name(tile, gram))
    rec = {
        "metric": "MI pair-updates/s (m*n(n+1)/2) & % int8 MFMA peak; p50/p99 request latency",
        "value": value,
        "unit": "pair-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "e2m1->f32" if gram == mi.MI_GRAM_FP4 else "int8",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "m": m, "n": n, "layout": "uint8 0/1 row-major, pitch %d" % X.stride(0),
            "density": "p_j log-uniform [0.001, 0.2]" if args.workload.startswith("large") else "see recipe",
            "epilogue": ["fp32", "fp32+fp64-fallback", "fp64"][args.epilogue],
            "tile": [None, 128, 256][tile], "splits": splits, "gram": GRAM_NAMES[gram],
            "conversion": conversion, "step_ms_on_stream": avg_step_s * 1e3,
        },
        "roofline": roofline(m, in_bytes, n, avg_kernel_s, achieved, traffic, tile, gram),
        # End to end (conversion included), 2 ops per pair-update, against the int8 peak.
        "frac_int8_peak": 2.0 * value / PEAK_INT8_OPS,
        "int8_kernel": int8_kernel,
    }
    del X
    torch.cuda.empty_cache()
    extras = set() if (args.no_extras or args.shape) else set(args.extras.split(","))
    rec.update(run_extras(dev, extras, args))
    if args.cpu_seconds > 0:
        rec["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
