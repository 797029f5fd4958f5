#!/usr/bin/env python3
"""Benchmark of the DFR sort hot path on one MI355X.

Workloads (``--workload``):

* ``plain`` (default) -- the headline configuration, below.
* ``batched`` -- 20,000 independent uint32 arrays with lengths log-uniform in
  [16, --max-len] (default 2^20) and a uint32 index payload, sorted by one segmented
  call after the autotuner has picked its launch settings on the same data; the same
  arrays sorted by one plain call each are timed beside it.
* ``serving`` -- a Poisson stream of sort requests (sizes log-uniform in
  [2^10, 2^24], 70% uint32 / 30% uint64 keys with a payload of the key's width,
  uniform or Zipf keys), offered at a load rho of the mean service time of one plain
  call (0.3 to 0.9, and 1.2 and 1.5 beyond what plain calls can serve), served (a) by
  FIFO plain calls on one stream and (b) by the context's request queue (dfr_submit /
  dfr_poll: continuous batching into segmented sorts) under a 32 GiB HBM budget.
  Latency is arrival to completion; p50/p99 and throughput for both.

Plain workload: one step = one plain DFR sort (count, deals of the top digits, bucket finding, local
sort of runs of small buckets, recursion if any) of 2^28 uint32 keys drawn i.i.d.
uniform over [0, 2^32) with a uint32 index payload, seed 0.  Every step sorts its own
copy of that input, made resident in HBM before the timed region starts, so the timed
region holds nothing but the sorts.

Printed: ONE JSON line with the throughput (Gkeys/s), the roofline of the dominant
kernel (the deal pass) from HIP events recorded around its launches during the timed
region, and the CPU oracle timed on a bounded sample of the same workload.
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


def cpu_baseline(dist, log2n_sample=24, seeds=(0, 1, 2)):
    """The CPU oracle (single-threaded C stable sort) on a bounded sample."""
    import oracle
    import workloads
    o = oracle.get()
    total_keys, total_s = 0, 0.0
    for seed in seeds:
        k = workloads.make_keys(dist, 1 << log2n_sample, 32, seed)
        v = workloads.index_payload(k.size)
        t0 = time.perf_counter()
        o.stable_sort(k, v)
        total_s += time.perf_counter() - t0
        total_keys += k.size
    return {
        "value": round(total_keys / total_s / 1e9, 5), "unit": "Gkeys/s", "cores": 1,
        "kind": "oracle",
        "sample": f"{len(seeds)} x 2^{log2n_sample} {dist} uint32 keys with uint32 index "
                  f"payload (seeds {list(seeds)}), single-threaded, {total_s:.1f} s",
    }


def copy_ceiling(torch, gib=4, reps=5):
    """The achievable HBM ceiling for comparison: a device-to-device copy of `gib` GiB
    by the runtime (read + write bytes over the copy's time, median of `reps`)."""
    import numpy as np
    n = (gib << 30) // 4
    src = torch.empty(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    t = float(np.median(ms))
    gbs = 2 * (gib << 30) / (t * 1e-3) / 1e9
    return {"bytes_copied": gib << 30, "ms": round(t, 4), "GB/s": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def check_segments(keys_in, keys_out, vals_out, off, segs):
    """check_result on the listed segments (payload = global index)."""
    for s in segs:
        a, b = int(off[s]), int(off[s + 1])
        r = check_result(keys_in[a:b], keys_out[a:b], vals_out[a:b] - vals_out.dtype.type(a))
        if r != "pass":
            return f"segment {s}: {r}"
    return "pass"


def run_batched(args):
    """Batched segmented sort against one plain call per array."""
    import numpy as np
    import torch

    import oracle
    import paper_2207_14334_amd as dfr
    import workloads

    torch.cuda.set_device(0)
    lens = workloads.batch_lengths(args.arrays, 16, args.max_len, 0)
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    log(f"generating {args.arrays} arrays, {n} {args.dist} keys")
    keys_h = workloads.make_keys(args.dist, n, 32, 0)
    vals_h = workloads.index_payload(n)
    base_k = torch.from_numpy(keys_h).cuda()
    base_v = torch.from_numpy(vals_h).cuda()
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
    log(f"autotune: {tune}")
    for _ in range(args.warmup):
        timed_segmented()
    times = [timed_segmented() for _ in range(args.steps)]
    ctx.set_option("timing", 1)
    timed_segmented()
    stages = ctx.stats()
    ctx.set_option("timing", 0)
    ms = float(np.median(times))
    gkeys = n / (ms * 1e-3) / 1e9
    log(f"segmented: median {ms:.2f} ms over {args.steps}, {gkeys:.2f} Gkeys/s")
    k_out, v_out = k.cpu().numpy(), v.cpu().numpy()
    rng = np.random.default_rng(1)
    sample = sorted(set(rng.integers(0, lens.size, 200).tolist()) | {int(np.argmax(lens))})
    parity = check_segments(keys_h, k_out, v_out, off, sample)
    log(f"result check on {len(sample)} segments: {parity}")
    del k_out, v_out

    # One plain call per array, on the same stream, the host waiting on nothing but
    # what each call itself waits for.
    plain = []
    for _ in range(args.plain_runs):
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
    log(f"plain calls: {plain_ms:.1f} ms, {n / plain_ms / 1e6:.3f} Gkeys/s")

    cpu = None
    if not args.no_cpu_baseline:
        o = oracle.get()
        m = int(np.searchsorted(off, 1 << 24))  # first arrays, about 2^24 keys
        t0 = time.perf_counter()
        o.segmented_sort(keys_h[: off[m]], vals_h[: off[m]], off[: m + 1])
        dt = time.perf_counter() - t0
        cpu = {"value": round(int(off[m]) / dt / 1e9, 5), "unit": "Gkeys/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the first {m} arrays ({int(off[m])} keys) of the same batch, "
                         f"single-threaded, {dt:.1f} s"}

    out = {
        "metric": METRIC, "value": round(gkeys, 4), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"batched segmented sort of {args.arrays} uint32 arrays, "
                               f"lengths log-uniform in [16, {args.max_len}], {args.dist} "
                               f"keys, uint32 index payload, seed 0",
                   "n": n, "arrays": int(lens.size), "max_len": args.max_len,
                   "distribution": args.dist, "parallelism": "single GPU"},
        "plain_calls": {"ms": round(plain_ms, 2), "gkeys_per_s": round(n / plain_ms / 1e6, 4),
                        "speedup_of_batched": round(plain_ms / ms, 2)},
        "tune": tune, "untuned_ms": round(tune["ms_default"], 4),
        "stage_ms": {kk: round(vv, 4) for kk, vv in stages.items() if kk.startswith("ms_")},
        "plan": {kk: stages[kk] for kk in ("levels", "top_digits", "deal_passes", "large_buckets")},
        "cpu_baseline": cpu,
        "result_check": parity,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    if parity != "pass":
        sys.exit(1)


def run_serving(args):
    """Poisson request stream: FIFO plain calls against the batching request queue."""
    import threading

    import numpy as np
    import torch

    import paper_2207_14334_amd as dfr
    import workloads

    torch.cuda.set_device(0)
    stream = workloads.request_stream(args.requests, 1.0, 1 << 10, 1 << 24, 0.3, 0.5, 0)
    unit_arrivals = np.array([a for a, _, _, _ in stream])  # at rate 1 per second
    log(f"generating {len(stream)} requests, {sum(r[1] for r in stream)} keys")
    from concurrent.futures import ThreadPoolExecutor

    def gen(i):
        _, n, bits, dist = stream[i]
        return workloads.make_keys(dist, n, bits, 1000 + i), workloads.index_payload(n, bits)

    base, work = [], []
    with ThreadPoolExecutor(8) as ex:  # numpy draws release the GIL
        for kh, vh in ex.map(gen, range(len(stream))):
            k = torch.from_numpy(kh).cuda()
            v = torch.from_numpy(vh).cuda()
            base.append((k, v))
            work.append((torch.empty_like(k), torch.empty_like(v)))
    total_keys = sum(r[1] for r in stream)
    torch.cuda.synchronize()

    def reset():
        for (bk, bv), (wk, wv) in zip(base, work):
            wk.copy_(bk)
            wv.copy_(bv)
        torch.cuda.synchronize()

    ctx = dfr.Context(0, hbm_budget_bytes=args.budget_gib << 30)
    # Mean service time of one plain call: the whole stream back to back.
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
    log(f"plain call: {svc_mean * 1e3:.3f} ms mean over the stream")

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
        submitted = threading.Event()
        t0 = time.perf_counter() + 0.01

        def submitter():
            for i, (k, v) in enumerate(work):
                spin_until(t0 + arrive[i])
                sub_delay[i] = time.perf_counter() - (t0 + arrive[i])
                tickets[i] = ctx.submit(k, v)
            submitted.set()

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

    # Warm the serving workers up as the plain calls were warmed up: the largest
    # requests of each width once, so that their buffers exist before the timed runs.
    reset()
    warm = []
    for bits in (32, 64):
        idx = [i for i, r in enumerate(stream) if r[2] == bits]
        for i in sorted(idx, key=lambda i: -stream[i][1])[:4]:
            warm.append(ctx.submit(*work[i]))
    for t in warm:
        while not ctx.poll(t)[0]:
            time.sleep(1e-4)
    out_rho = {}
    st0 = ctx.serve_stats()
    for rho in args.rho:
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
        out_rho[str(rho)] = r
        log(f"rho {rho}: {json.dumps(r)}")

    # Results of the last served run: each request sorted (properties of the stable
    # sort under the index payload) on a sample.
    rng = np.random.default_rng(3)
    parity = "pass"
    for i in sorted(set(rng.integers(0, len(work), 40).tolist())):
        kin = base[i][0].cpu().numpy()
        r = check_result(kin, work[i][0].cpu().numpy(), work[i][1].cpu().numpy())
        if r != "pass":
            parity = f"request {i}: {r}"
            break
    head = out_rho[str(args.rho[-1] if 0.7 not in args.rho else 0.7)]
    out = {
        "metric": METRIC, "value": head["served"]["gkeys_per_s"], "unit": "Gkeys/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64", "data": "synthetic",
        "config": {"workload": f"serving: {len(stream)} Poisson sort requests, sizes log-uniform "
                               f"in [2^10, 2^24], 70% uint32 / 30% uint64 keys with payload, "
                               f"50% uniform / 50% Zipf, HBM budget {args.budget_gib} GiB",
                   "requests": len(stream), "keys": total_keys,
                   "plain_call_ms_mean": round(svc_mean * 1e3, 4), "headline_rho": 0.7,
                   "parallelism": "single GPU"},
        "p50_ms": head["served"]["p50_ms"], "p99_ms": head["served"]["p99_ms"],
        "p99_plain_fifo_ms": head["fifo_plain"]["p99_ms"],
        "by_rho": out_rho, "serve_stats": ctx.serve_stats(), "result_check": parity,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    if parity != "pass":
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("plain", "batched", "serving"), default="plain")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rho", type=float, nargs="+", default=[0.3, 0.5, 0.7, 0.9, 1.2, 1.5])
    ap.add_argument("--budget-gib", type=int, default=32)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--dist", default="uniform")
    ap.add_argument("--arrays", type=int, default=20000)
    ap.add_argument("--max-len", type=int, default=1 << 20)
    ap.add_argument("--plain-runs", type=int, default=2)
    ap.add_argument("--key-type", default="u32", choices=("u32", "u64", "i32", "i64", "f32", "f64"))
    ap.add_argument("--set", action="append", default=[], metavar="OPTION=VALUE",
                    help="a library option (dfr_set_option) for the plain workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip the runtime copy timing (profiling runs calibrate on the input copies)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the sort's "
                                   "multi-GPU path (histogram all-reduce, splitters, "
                                   "all-to-all exchange) is not built"}), flush=True)
        sys.exit(2)
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "serving":
        return run_serving(args)
    return run_plain(args)


def run_plain(args):
    import numpy as np
    import torch

    import paper_2207_14334_amd as dfr
    import workloads

    torch.cuda.set_device(0)
    n = 1 << args.log2n
    kt = args.key_type
    kbits = 32 if kt.endswith("32") else 64
    kb = vb = kbits // 8
    log(f"generating {n} {args.dist} {kt} keys")
    # Signed and float keys are the same seeded bit patterns viewed as that type.
    bits_h = workloads.make_keys(args.dist, n, kbits, 0)
    keys_h = bits_h.view({"u32": np.uint32, "u64": np.uint64, "i32": np.int32, "i64": np.int64,
                          "f32": np.float32, "f64": np.float64}[kt])
    vals_h = workloads.index_payload(n, kbits)
    base_k = torch.from_numpy(keys_h).cuda()
    base_v = torch.from_numpy(vals_h).cuda()
    copies = args.warmup + args.steps
    ks = [torch.empty_like(base_k) for _ in range(copies)]
    vs = [torch.empty_like(base_v) for _ in range(copies)]
    for i in range(copies):
        ks[i].copy_(base_k)
        vs[i].copy_(base_v)
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
    ks[0].copy_(base_k)
    vs[0].copy_(base_v)
    ctx.set_option("timing", 1)
    ctx.sort_(ks[0], vs[0], temp)
    torch.cuda.synchronize()
    stage = ctx.stats()
    ctx.set_option("timing", 0)
    # Cold variant: the first sort on a fresh context, its scratch (temp buffer, arena,
    # pinned staging) allocated inside the call, as a one-off caller would see it.
    ks[0].copy_(base_k)
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
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, {gkeys:.2f} Gkeys/s")

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

    parity = check_result(as_ordered(keys_h), as_ordered(ks[-1].cpu().numpy()), vs[-1].cpu().numpy())
    log(f"result check: {parity}")

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

    cpu = None if args.no_cpu_baseline or kt != "u32" else cpu_baseline(args.dist)
    ceiling = None if args.no_copy_ceiling else copy_ceiling(torch)

    out = {
        "metric": METRIC, "value": round(gkeys, 4), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": kt,
        "data": "synthetic",
        "config": {"workload": f"plain DFR sort of 2^{args.log2n} {kt} keys, i.i.d. "
                               f"{args.dist} bit patterns, uint{kbits} index payload, seed 0",
                   "n": n, "key_type": kt, "key_bits": kbits, "payload_bits": kbits,
                   "distribution": args.dist, "options": args.set,
                   "parallelism": "single GPU"},
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
        "stage_ms_one_sort": {k: round(v, 4) for k, v in stage.items() if k.startswith("ms_")},
        "cold_first_sort_ms": round(cold_ms, 3),
        "step_ms": {"median": round(float(np.median(step_ms)), 4),
                    "min": round(float(step_ms.min()), 4),
                    "p90": round(float(np.percentile(step_ms, 90)), 4)},
        "copy_ceiling": ceiling,
        "result_check": parity,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    if parity != "pass":
        sys.exit(1)


if __name__ == "__main__":
    main()
