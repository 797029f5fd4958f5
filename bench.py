#!/usr/bin/env python3
"""Benchmark of the DFR sort hot path on one MI355X.

Default run (``--workload all``): one JSON line whose headline is the plain sort below,
with the rest of the metric beside it:

* ``value`` -- plain DFR sort of 2^28 uint32 keys, i.i.d. uniform over [0, 2^32), with a
  uint32 index payload; every step sorts its own resident copy of one of three inputs
  (seeds 0, 1, 2, in turn), and ``value`` is the keys sorted over the timed steps' time.
  Per-seed rates are in ``value_by_seed``.
* ``roofline`` -- the deal kernel (the dominant pass): algorithmic bytes per launch over
  its mean launch time from HIP events on the sort's stream during the timed steps;
  ``copy_ceiling`` -- the library's own streaming copy kernel on 4 GiB, the rate the
  read-once/write-once passes can reach; ``read_ceiling`` -- its streaming read kernel
  on 1 GiB (the 2^28 uint32 keys a count reads), the rate a count can reach.
* ``cpu_baseline`` -- the CPU oracle on the host: all cores on the full 2^28 input of
  seed 0, and single-threaded on three 2^24 samples.
* ``c1`` -- 2^20 uint32 keys, key-only: wall latency of one call.
* ``normal`` -- the 2^28 sort on the normal distribution (mean 2^31, sd 2^28).
* ``batched`` -- 20,000 uint32 arrays, lengths log-uniform in [16, 2^20] (1.9e9 keys),
  uniform and Zipf(1.1) keys with the global index as payload: one tuned segmented call
  against one plain call per array, with a per-segment check of sampled arrays.
* ``serving`` -- 2,000 Poisson sort requests (sizes log-uniform in [2^10, 2^24], 70%
  uint32 / 30% uint64 keys with a payload of the key's width, half uniform, half Zipf)
  at offered loads 0.7 and 0.9 of one plain call's mean service time: FIFO plain calls
  against the request queue's continuous batching, p50/p99 latency and throughput.

``--workload plain|batched|serving`` runs one part alone (the first with --log2n,
--dist, --key-type and --set OPTION=VALUE for other shapes); batched and serving inputs
are drawn on the GPU (seeded), the plain inputs with numpy.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gkeys/s at 2^28 u32 & % HBM peak; batched/serving p99 vs plain calls"
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "deal_u32x32_2p28_uniform_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2207_14334_amd", "csrc", "kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_traffic():
    """Per-launch HBM bytes of the deal kernel from the committed rocprofv3 counter
    summary, or None if that summary is missing or was taken on other kernel source."""
    try:
        text = open(PROFILE_COUNTERS).read()
    except OSError:
        return None
    m_hash = re.search(r"kernels\.hip sha256:\s*([0-9a-f]{64})", text)
    m_bytes = re.search(r"traffic bytes per launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def check_result(keys_in, keys_out, vals_out):
    """Stable-sort properties under the index payload (numpy, no oracle)."""
    import numpy as np
    n = keys_in.size
    if not (keys_out[1:] >= keys_out[:-1]).all():
        return "keys not sorted"
    if np.bincount(vals_out.astype(np.int64), minlength=n).max() != 1:
        return "payload is not a permutation"
    if not np.array_equal(keys_in[vals_out], keys_out):
        return "key/payload mismatch"
    eq = keys_out[1:] == keys_out[:-1]
    if not (vals_out[1:][eq] > vals_out[:-1][eq]).all():
        return "equal keys out of input order"
    return "pass"


def cpu_baseline(keys_full, dist="uniform", log2n_sample=24, seeds=(0, 1, 2)):
    """The CPU oracle on the host: all cores (chunked stable sort, then a stable merge
    tree) on the full input, and one thread on bounded samples of the same workload."""
    import numpy as np

    import oracle
    import workloads
    o = oracle.get()
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    threads = max(1, min(16, cores))
    vals = workloads.index_payload(keys_full.size)
    t0 = time.perf_counter()
    o.stable_sort_parallel(keys_full, vals, threads)
    par_s = time.perf_counter() - t0
    del vals
    total_keys, total_s = 0, 0.0
    for seed in seeds:
        k = workloads.make_keys(dist, 1 << log2n_sample, 32, seed)
        v = workloads.index_payload(k.size)
        t0 = time.perf_counter()
        o.stable_sort(k, v)
        total_s += time.perf_counter() - t0
        total_keys += k.size
    return {
        "value": round(keys_full.size / par_s / 1e9, 5), "unit": "Gkeys/s", "cores": threads,
        "kind": "oracle",
        "sample": f"the full 2^{int(np.log2(keys_full.size))} {dist} uint32 input of seed 0 with "
                  f"its uint32 index payload, {threads} threads (chunks sorted by (key, index), "
                  f"then a stable pairwise merge tree), {par_s:.1f} s",
        "hardware_concurrency": os.cpu_count(),
        "single_thread": {
            "value": round(total_keys / total_s / 1e9, 5), "unit": "Gkeys/s", "cores": 1,
            "sample": f"{len(seeds)} x 2^{log2n_sample} {dist} uint32 keys with uint32 index "
                      f"payload (seeds {list(seeds)}), {total_s:.1f} s"},
    }


def copy_ceiling(torch, ctx, gib=4, reps=5):
    """The library's streaming copy kernel on `gib` GiB (read + write bytes over its time
    from HIP events on its stream, median of `reps`): what a pass that reads and writes
    every byte once can reach on this GPU."""
    import numpy as np
    n = (gib << 30) // 4
    src = torch.empty(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    ctx.stream_copy(src, dst)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.stream_copy(src, dst)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    ok = bool(torch.equal(src, dst))
    del src, dst
    torch.cuda.empty_cache()
    t = float(np.median(ms))
    gbs = 2 * (gib << 30) / (t * 1e-3) / 1e9
    return {"kernel": "k_stream_copy", "bytes_copied": gib << 30, "ms": round(t, 4),
            "GB/s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "copy_correct": ok}


def read_ceiling(torch, ctx, gib=1, reps=5):
    """The library's streaming read kernel on `gib` GiB of random words (bytes read over
    its time from HIP events on its stream, median of `reps`), with its XOR checksum
    checked against a fold of the same words by torch's own XOR."""
    import numpy as np
    n = (gib << 30) // 4
    src = torch.randint(-(1 << 31), (1 << 31) - 1, (n,), dtype=torch.int32, device="cuda")
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.stream_read(src, out)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.stream_read(src, out)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    x = src
    while x.numel() > 1:  # n is a power of two
        h = x.numel() // 2
        x = torch.bitwise_xor(x[:h], x[h:])
    ok = bool(torch.equal(x, out))
    del src, out, x
    torch.cuda.empty_cache()
    t = float(np.median(ms))
    gbs = (gib << 30) / (t * 1e-3) / 1e9
    return {"kernel": "k_stream_read", "bytes_read": gib << 30, "ms": round(t, 4),
            "GB/s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "checksum_correct": ok}


def check_segments(keys_in, keys_out, vals_out, off, segs):
    """check_result on the listed segments (payload = global index)."""
    for s in segs:
        a, b = int(off[s]), int(off[s + 1])
        r = check_result(keys_in[a:b], keys_out[a:b], vals_out[a:b] - vals_out.dtype.type(a))
        if r != "pass":
            return f"segment {s}: {r}"
    return "pass"


def host_np(t):
    """A uint32/uint64 GPU tensor as a numpy array of the same unsigned type."""
    import numpy as np
    import torch
    if t.dtype == torch.uint32:
        return t.view(torch.int32).cpu().numpy().view(np.uint32)
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def batched_part(torch, dfr, dist, arrays, max_len, steps, plain_runs=1):
    """One tuned segmented call over the batch against one plain call per array."""
    import numpy as np

    import workloads
    lens = workloads.batch_lengths(arrays, 16, max_len, 0)
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    log(f"batched {dist}: drawing {n} keys on the GPU")
    base_k = workloads.make_keys_device(dist, n, 32, 0)
    base_v = workloads.index_payload_device(n, 32)
    k = torch.empty_like(base_k)
    v = torch.empty_like(base_v)
    temp = torch.empty(dfr.temp_bytes(n, 4, 4), dtype=torch.uint8, device="cuda")
    ctx = dfr.Context(0)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed_segmented():
        k.copy_(base_k)
        v.copy_(base_v)
        ev[0].record(stream)
        ctx.sort_segmented_(k, v, off, temp)
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1])

    tune = ctx.autotune(base_k, base_v, off, reps=1)
    log(f"batched {dist}: autotune {tune}")
    timed_segmented()
    times = [timed_segmented() for _ in range(steps)]
    st = ctx.stats()
    ms = float(np.median(times))
    gkeys = n / (ms * 1e-3) / 1e9
    log(f"batched {dist}: segmented median {ms:.2f} ms, {gkeys:.2f} Gkeys/s")
    rng = np.random.default_rng(1)
    sample = sorted(set(rng.integers(0, lens.size, 200).tolist()) | {int(np.argmax(lens))})
    kin_h, kout_h, vout_h = host_np(base_k), host_np(k), host_np(v)
    parity = check_segments(kin_h, kout_h, vout_h, off, sample)
    del kin_h, kout_h, vout_h
    log(f"batched {dist}: check of {len(sample)} segments: {parity}")
    plain = []
    for _ in range(plain_runs):
        k.copy_(base_k)
        v.copy_(base_v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(lens.size):
            a, b = int(off[i]), int(off[i + 1])
            ctx.sort_(k[a:b], v[a:b], temp)
        torch.cuda.synchronize()
        plain.append((time.perf_counter() - t0) * 1e3)
    plain_ms = min(plain)
    log(f"batched {dist}: plain calls {plain_ms:.1f} ms")
    ctx.close()
    del base_k, base_v, k, v, temp
    torch.cuda.empty_cache()
    return {
        "workload": f"{arrays} uint32 arrays, lengths log-uniform in [16, {max_len}], {dist} keys, "
                    f"uint32 global-index payload, seed 0",
        "n": n, "segmented_ms": round(ms, 3), "gkeys_per_s": round(gkeys, 3),
        "untuned_ms": round(tune["ms_default"], 3),
        "tune": {kk: tune[kk] for kk in ("radix_bits", "tile_records", "divert_records", "window_records")},
        "plain_calls_ms": round(plain_ms, 1),
        "plain_calls_gkeys_per_s": round(n / plain_ms / 1e6, 4),
        "speedup_over_plain_calls": round(plain_ms / ms, 1),
        "plan": {kk: st[kk] for kk in ("levels", "top_digits", "deal_passes", "large_buckets")},
        "result_check": parity, "segments_checked": len(sample),
    }


def serving_part(torch, dfr, requests, rhos, budget_gib, options=()):
    """Poisson request stream: FIFO plain calls against the batching request queue
    (library options (name, value) set on its context before the first request)."""
    import threading

    import numpy as np

    import workloads
    stream_def = workloads.request_stream(requests, 1.0, 1 << 10, 1 << 24, 0.3, 0.5, 0)
    unit_arrivals = np.array([a for a, _, _, _ in stream_def])  # at rate 1 per second
    total_keys = sum(r[1] for r in stream_def)
    log(f"serving: drawing {len(stream_def)} requests, {total_keys} keys on the GPU")
    base, work = [], []
    for i, (_, n, bits, dist) in enumerate(stream_def):
        k = workloads.make_keys_device(dist, n, bits, 1000 + i)
        v = workloads.index_payload_device(n, bits)
        base.append((k, v))
        work.append((torch.empty_like(k), torch.empty_like(v)))
    torch.cuda.synchronize()

    def reset():
        for (bk, bv), (wk, wv) in zip(base, work):
            wk.copy_(bk)
            wv.copy_(bv)
        torch.cuda.synchronize()

    ctx = dfr.Context(0, hbm_budget_bytes=budget_gib << 30)
    for name, value in options:
        ctx.set_option(name, value)
    sys.setswitchinterval(2e-4)  # the submitting thread must not wait long for the GIL
    reset()
    for i in range(min(len(work), 30)):
        ctx.sort_(*work[i])
    reset()
    t0 = time.perf_counter()
    for k, v in work:
        ctx.sort_(k, v)
    torch.cuda.synchronize()
    svc_mean = (time.perf_counter() - t0) / len(work)
    log(f"serving: plain call {svc_mean * 1e3:.3f} ms mean over the stream")

    def spin_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            if d > 2e-4:
                time.sleep(d - 1e-4)

    def fifo(arrive):
        reset()
        lat = np.zeros(len(work))
        t0 = time.perf_counter() + 0.01
        done = 0.0
        for i, (k, v) in enumerate(work):
            spin_until(t0 + arrive[i])
            ctx.sort_(k, v)
            done = time.perf_counter()
            lat[i] = done - (t0 + arrive[i])
        return lat, done - t0

    def served(arrive):
        reset()
        n = len(work)
        tickets = [None] * n
        sub_delay = np.zeros(n)
        lat = np.full(n, np.nan)
        t0 = time.perf_counter() + 0.01

        def submitter():
            for i, (k, v) in enumerate(work):
                spin_until(t0 + arrive[i])
                sub_delay[i] = time.perf_counter() - (t0 + arrive[i])
                tickets[i] = ctx.submit(k, v)

        th = threading.Thread(target=submitter)
        th.start()
        left = set()
        nxt = 0
        while nxt < n or left:
            while nxt < n and tickets[nxt] is not None:
                left.add(nxt)
                nxt += 1
            for i in list(left):
                ok, l = ctx.poll(tickets[i])
                if ok:
                    lat[i] = l + sub_delay[i]
                    left.discard(i)
            time.sleep(2e-4)
        th.join()
        end = max(arrive[i] + lat[i] for i in range(n))
        return lat, end

    # Warm the workers up as the plain calls were (these ran the whole stream once): one
    # untimed served pass of the whole stream at the highest load, so that every worker's
    # buffers have grown to their working size before the timed runs.
    served(unit_arrivals * svc_mean / max(rhos))
    by_rho = {}
    st0 = ctx.serve_stats()
    for rho in rhos:
        arrive = unit_arrivals * svc_mean / rho
        lat_p, span_p = fifo(arrive)
        lat_s, span_s = served(arrive)
        st = ctx.serve_stats()
        r = {
            "offered_rate_per_s": round(rho / svc_mean, 1),
            "fifo_plain": {"p50_ms": round(float(np.percentile(lat_p, 50)) * 1e3, 3),
                           "p99_ms": round(float(np.percentile(lat_p, 99)) * 1e3, 3),
                           "gkeys_per_s": round(total_keys / span_p / 1e9, 3)},
            "served": {"p50_ms": round(float(np.percentile(lat_s, 50)) * 1e3, 3),
                       "p99_ms": round(float(np.percentile(lat_s, 99)) * 1e3, 3),
                       "gkeys_per_s": round(total_keys / span_s / 1e9, 3),
                       "batches": st["batches"] - st0["batches"],
                       "max_batch_requests": st["max_batch_requests"]},
        }
        r["p99_ratio_plain_over_served"] = round(r["fifo_plain"]["p99_ms"] / r["served"]["p99_ms"], 3)
        st0 = st
        by_rho[str(rho)] = r
        log(f"serving rho {rho}: {json.dumps(r)}")
    # The last served run's results: each sampled request sorted (the stable sort's
    # properties under the index payload).
    rng = np.random.default_rng(3)
    parity = "pass"
    for i in sorted(set(rng.integers(0, len(work), 40).tolist())):
        r = check_result(host_np(base[i][0]), host_np(work[i][0]), host_np(work[i][1]))
        if r != "pass":
            parity = f"request {i}: {r}"
            break
    out = {
        "workload": f"{len(stream_def)} Poisson sort requests, sizes log-uniform in [2^10, 2^24], "
                    f"70% uint32 / 30% uint64 keys with a payload of the key's width, 50% uniform / "
                    f"50% Zipf(1.1), HBM budget {budget_gib} GiB",
        "requests": len(stream_def), "keys": total_keys,
        "plain_call_ms_mean": round(svc_mean * 1e3, 4), "by_rho": by_rho,
        "serve_stats": {kk: vv for kk, vv in ctx.serve_stats().items()
                        if kk in ("batches", "requests", "max_batch_requests", "peak_held_bytes",
                                  "allocs")},
        "options": [f"{name}={value}" for name, value in options],
        "result_check": parity, "requests_checked": 40,
    }
    ctx.close()
    del base, work
    torch.cuda.empty_cache()
    return out


def c1_part(torch, dfr, calls=50, options=()):
    """2^20 uint32 keys, key-only (small enough to stay in the caches): wall time of one
    call, from its start to the end of its work on the stream."""
    import numpy as np

    import workloads
    n = 1 << 20
    keys_h = workloads.make_keys("uniform", n, 32, 0)
    base = torch.from_numpy(keys_h).cuda()
    copies = [base.clone() for _ in range(calls + 5)]
    ctx = dfr.Context(0)
    for name, value in options:
        ctx.set_option(name, value)
    torch.cuda.synchronize()
    for i in range(5):
        ctx.sort_(copies[i])
    torch.cuda.synchronize()
    wall = []
    for i in range(5, calls + 5):
        t0 = time.perf_counter()
        ctx.sort_(copies[i])
        torch.cuda.synchronize()
        wall.append((time.perf_counter() - t0) * 1e3)
    st = ctx.stats()
    ok = np.array_equal(host_np(copies[-1]), np.sort(keys_h))
    ctx.close()
    w = np.array(wall)
    opts = "".join(f", option {name}={value}" for name, value in options)
    return {"workload": f"2^20 uint32 keys, uniform, key-only, seed 0{opts}", "n": n,
            "latency_ms": {"median": round(float(np.median(w)), 4), "min": round(float(w.min()), 4),
                           "p90": round(float(np.percentile(w, 90)), 4)},
            "gkeys_per_s": round(n / np.median(w) / 1e6, 3), "calls": calls,
            "plan": {kk: st[kk] for kk in ("levels", "top_digits", "deal_passes")},
            "result_check": "pass" if ok else "keys differ from numpy's sort"}


def dist_part(torch, dfr, dist, log2n=28, steps=3, options=()):
    """The plain 2^log2n uint32 + index payload sort on another distribution, or under
    library options (name, value)."""
    import numpy as np

    import workloads
    n = 1 << log2n
    keys_h = workloads.make_keys(dist, n, 32, 0)
    base_k = torch.from_numpy(keys_h).cuda()
    base_v = torch.from_numpy(workloads.index_payload(n)).cuda()
    k, v = torch.empty_like(base_k), torch.empty_like(base_v)
    temp = torch.empty(dfr.temp_bytes(n, 4, 4), dtype=torch.uint8, device="cuda")
    ctx = dfr.Context(0)
    for name, value in options:
        ctx.set_option(name, value)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for i in range(steps + 1):
        k.copy_(base_k)
        v.copy_(base_v)
        ev[0].record()
        ctx.sort_(k, v, temp)
        ev[1].record()
        torch.cuda.synchronize()
        if i:
            times.append(ev[0].elapsed_time(ev[1]))
    st = ctx.stats()
    parity = check_result(keys_h, host_np(k), host_np(v))
    ctx.set_option("timing", 1)
    k.copy_(base_k)
    v.copy_(base_v)
    ctx.sort_(k, v, temp)
    torch.cuda.synchronize()
    stages = {kk: round(vv, 4) for kk, vv in ctx.stats().items() if kk.startswith("ms_")}
    ctx.close()
    del base_k, base_v, k, v, temp
    torch.cuda.empty_cache()
    ms = float(np.median(times))
    opts = "".join(f", option {name}={value}" for name, value in options)
    return {"workload": f"2^{log2n} uint32 keys, {dist}, uint32 index payload, seed 0{opts}", "n": n,
            "ms": round(ms, 4), "gkeys_per_s": round(n / ms / 1e6, 3),
            "plan": {kk: st[kk] for kk in ("levels", "top_digits", "deal_passes", "large_buckets",
                                           "deal_passes_estimated", "estimated_overflow")},
            "stage_ms": stages, "result_check": parity}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=("all", "plain", "batched", "serving"), default="all")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rho", type=float, nargs="+", default=None,
                    help="offered loads of the serving part (default 0.7 0.9; alone 0.3 .. 1.5)")
    ap.add_argument("--budget-gib", type=int, default=32)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--dist", default="uniform")
    ap.add_argument("--arrays", type=int, default=20000)
    ap.add_argument("--max-len", type=int, default=1 << 20)
    ap.add_argument("--key-type", default="u32", choices=("u32", "u64", "i32", "i64", "f32", "f64"))
    ap.add_argument("--set", action="append", default=[], metavar="OPTION=VALUE",
                    help="a library option (dfr_set_option) for the plain or serving workload")
    ap.add_argument("--seeds", type=int, default=3, help="inputs the plain steps cycle through")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip the copy and read reference timings (profiling runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the sort's "
                                   "multi-GPU path (histogram all-reduce, splitters, "
                                   "all-to-all exchange) is not built"}), flush=True)
        sys.exit(2)
    import torch

    import paper_2207_14334_amd as dfr
    torch.cuda.set_device(0)
    wall0 = time.perf_counter()
    if args.workload == "batched":
        out = {"batched": [batched_part(torch, dfr, d, args.arrays, args.max_len, args.steps, 2)
                           for d in (("uniform", "zipf") if args.dist == "uniform" else (args.dist,))]}
        print(json.dumps(out), flush=True)
        return
    if args.workload == "serving":
        rhos = args.rho or [0.3, 0.5, 0.7, 0.9, 1.2, 1.5]
        opts = [(o.split("=", 1)[0], int(o.split("=", 1)[1])) for o in args.set]
        print(json.dumps({"serving": serving_part(torch, dfr, args.requests, rhos, args.budget_gib,
                                                  opts)}), flush=True)
        return
    out = run_plain(args, torch, dfr)
    ok = out["result_check"] == "pass"
    if args.workload == "all":
        out["c1"] = c1_part(torch, dfr)
        log(f"c1: {out['c1']}")
        # The same with the plan taken from the length alone: no read-back before the deal.
        out["c1_plan_from_length"] = c1_part(torch, dfr, options=[("plan_lengths_records", 1 << 22)])
        log(f"c1 plan from length: {out['c1_plan_from_length']}")
        out["normal"] = dist_part(torch, dfr, "normal")
        log(f"normal: {out['normal']}")
        # Fast Radix's estimated buckets for the first deal (no count) on the headline
        # input, against the counted path that "value" times.
        out["estimated_buckets"] = dist_part(torch, dfr, "uniform", options=[("estimated_buckets", 1)])
        log(f"estimated buckets: {out['estimated_buckets']}")
        out["batched"] = [batched_part(torch, dfr, d, args.arrays, args.max_len, 3)
                          for d in ("uniform", "zipf")]
        out["serving"] = serving_part(torch, dfr, args.requests, args.rho or [0.7, 0.9],
                                      args.budget_gib)
        ok = ok and all(p["result_check"] == "pass" for p in
                        [out["c1"], out["c1_plan_from_length"], out["normal"],
                         out["estimated_buckets"], out["serving"], *out["batched"]])
    out["wall_s"] = round(time.perf_counter() - wall0, 1)
    print(json.dumps(out), flush=True)
    if not ok:
        sys.exit(1)


def run_plain(args, torch, dfr):
    import numpy as np

    import workloads

    n = 1 << args.log2n
    kt = args.key_type
    kbits = 32 if kt.endswith("32") else 64
    kb = vb = kbits // 8
    seeds = list(range(max(1, args.seeds)))
    log(f"generating {len(seeds)} x {n} {args.dist} {kt} keys")
    # Signed and float keys are the same seeded bit patterns viewed as that type.
    view = {"u32": np.uint32, "u64": np.uint64, "i32": np.int32, "i64": np.int64,
            "f32": np.float32, "f64": np.float64}[kt]
    keys_h = [workloads.make_keys(args.dist, n, kbits, sd).view(view) for sd in seeds]
    vals_h = workloads.index_payload(n, kbits)
    base_k = [torch.from_numpy(kh).cuda() for kh in keys_h]
    base_v = torch.from_numpy(vals_h).cuda()
    copies = args.warmup + args.steps
    seed_of = [i % len(seeds) for i in range(copies)]
    ks = [base_k[seed_of[i]].clone() for i in range(copies)]
    vs = [base_v.clone() for _ in range(copies)]
    temp = torch.empty(dfr.temp_bytes(n, kb, vb), dtype=torch.uint8, device="cuda")
    ctx = dfr.Context(0)
    for opt in args.set:
        name, value = opt.split("=", 1)
        ctx.set_option(name, int(value))
    torch.cuda.synchronize()
    log(f"{copies} resident copies ready")

    for i in range(args.warmup):
        ctx.sort_(ks[i], vs[i], temp)
    torch.cuda.synchronize()
    log("warmup done")

    # Timed region: HIP events around the deal launches only (timing level 2), on the
    # sort's stream, for the roofline of the deal kernel.
    ctx.set_option("timing", 2)
    agg = {"ms_deal": 0.0, "deal_launches_timed": 0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = None
    stamps = [t0]
    for i in range(args.warmup, copies):
        ctx.sort_(ks[i], vs[i], temp)  # returns once the sort's last read-back is in
        stamps.append(time.perf_counter())
        st = ctx.stats()
        for k in agg:
            agg[k] += st[k]
        plan = st
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = np.diff(np.array(stamps)) * 1e3
    ctx.set_option("timing", 0)
    # Per-stage kernel times from one more sort after the timed region (events around
    # every stage add gaps between kernels, so they stay out of the timed steps).
    ks[0].copy_(base_k[0])
    vs[0].copy_(base_v)
    ctx.set_option("timing", 1)
    ctx.sort_(ks[0], vs[0], temp)
    torch.cuda.synchronize()
    stage = ctx.stats()
    ctx.set_option("timing", 0)
    # Cold variant: the first sort on a fresh context, its scratch (temp buffer, arena)
    # allocated inside the call, as a one-off caller would see it.
    ks[0].copy_(base_k[0])
    vs[0].copy_(base_v)
    torch.cuda.synchronize()
    cold_ctx = dfr.Context(0)
    c0 = time.perf_counter()
    cold_ctx.sort_(ks[0], vs[0])
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - c0) * 1e3
    cold_ctx.close()
    elapsed = t1 - t0
    ms_step = elapsed / args.steps * 1e3
    gkeys = n * args.steps / elapsed / 1e9
    by_seed = {}
    for sd in seeds:
        mine = [step_ms[j] for j in range(args.steps) if seed_of[args.warmup + j] == sd]
        if mine:
            by_seed[str(sd)] = round(n / (np.mean(mine) * 1e-3) / 1e9, 4)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, {gkeys:.2f} Gkeys/s, by seed {by_seed}")

    # The check compares the keys as unsigned integers of the same order: the encodings
    # themselves for unsigned keys, the sign bit flipped for signed ones, and for floats
    # every bit of a negative encoding or the sign bit of a positive one (totalOrder).
    def as_ordered(a):
        raw = a.view(np.uint32 if kbits == 32 else np.uint64)
        sign = raw.dtype.type(1 << (kbits - 1))
        if kt[0] == "i":
            return raw ^ sign
        if kt[0] == "f":
            neg = (raw & sign) != 0
            return np.where(neg, ~raw, raw ^ sign)
        return raw

    parity = "pass"
    for i in range(copies - len(seeds), copies):  # the last step of every seed
        r = check_result(as_ordered(keys_h[seed_of[i]]), as_ordered(ks[i].cpu().numpy()),
                         vs[i].cpu().numpy())
        if r != "pass":
            parity = f"seed {seed_of[i]}: {r}"
            break
    log(f"result check: {parity}")
    del ks, vs
    torch.cuda.empty_cache()

    rec_bytes = kb + vb
    deal_bytes = 2 * rec_bytes * n  # read + write of key and payload, one pass
    deal_ms = agg["ms_deal"] / max(agg["deal_launches_timed"], 1)
    deal_gbs = deal_bytes / (deal_ms * 1e-3) / 1e9
    headline = kt == "u32" and args.log2n == 28 and args.dist == "uniform" and not args.set
    traffic = counter_traffic() if headline else None
    # Algorithmic bytes of the whole sort: count (kb/key), d deals (2(kb+vb)/key),
    # bucket heads (kb/key), local sort (2(kb+vb)/key).
    d = plan["top_digits"] if plan else 0
    sort_bytes = n * (kb + d * 2 * rec_bytes + (kb + 2 * rec_bytes if plan and plan["used_diversion"] else 0))
    hbm_frac_sort = sort_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    cpu = None if args.no_cpu_baseline or kt != "u32" else cpu_baseline(keys_h[0], args.dist)
    if cpu:
        log(f"cpu baseline: {cpu}")
    del base_k, base_v, temp
    torch.cuda.empty_cache()
    ceiling = None if args.no_copy_ceiling else copy_ceiling(torch, ctx)
    rceiling = None if args.no_copy_ceiling else read_ceiling(torch, ctx)
    stage_ms = {k: round(v, 4) for k, v in stage.items() if k.startswith("ms_")}
    out = {
        "metric": METRIC, "value": round(gkeys, 4), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": kt,
        "data": "synthetic",
        "config": {"workload": f"plain DFR sort of 2^{args.log2n} {kt} keys, i.i.d. "
                               f"{args.dist} bit patterns, uint{kbits} index payload, seeds "
                               f"{seeds} in turn",
                   "n": n, "key_type": kt, "key_bits": kbits, "payload_bits": kbits,
                   "distribution": args.dist, "seeds": seeds, "options": args.set,
                   "parallelism": "single GPU"},
        "value_by_seed": by_seed,
        "roofline": {"bound": "hbm",
                     "kernel": f"k_deal<{kb},{vb},512,{dfr.deal_tile_records(kb, vb) // 512}>",
                     "achieved": round(deal_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(deal_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes_per_launch": deal_bytes,
                     "avg_launch_ms": round(deal_ms, 4),
                     "launches": agg["deal_launches_timed"]},
        "cpu_baseline": cpu,
        "hbm_frac_sort": round(hbm_frac_sort, 4),
        "plan": {"top_digits": d, "levels": plan["levels"] if plan else 0,
                 "deal_passes": plan["deal_passes"] if plan else 0,
                 "large_buckets": plan["large_buckets"] if plan else 0,
                 "estimated_bucket_overflow": plan["estimated_overflow"] if plan else None},
        "stage_ms_one_sort": stage_ms,
        "stage_frac_of_peak": {
            k: round(b / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            for k, b in (("ms_deal", d * 2 * rec_bytes * n),
                         ("ms_local_sort", 2 * rec_bytes * n if plan and plan["used_diversion"] else 0),
                         ("ms_count", kb * n * (1 + max(d - 1, 0))))
            if b and stage_ms.get(k)},
        "cold_first_sort_ms": round(cold_ms, 3),
        "step_ms": {"median": round(float(np.median(step_ms)), 4),
                    "min": round(float(step_ms.min()), 4),
                    "p90": round(float(np.percentile(step_ms, 90)), 4)},
        "copy_ceiling": ceiling,
        "read_ceiling": rceiling,
        "result_check": parity,
    }
    ctx.close()
    return out


if __name__ == "__main__":
    main()
