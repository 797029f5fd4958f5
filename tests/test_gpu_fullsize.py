"""GPU parity at the benchmark's full sizes, in the configuration bench.py times.

2^28 uint32 keys with a uint32 index payload on each key distribution of that workload
(uniform, normal, Zipf, sorted, reverse-sorted, 256 distinct values), and 2^27 uint64
keys with a uint64 index payload (uniform, and top-16-bits-from-4-values skewed); and the
batched segmented sort of 20,000 uint32 arrays with lengths log-uniform in [16, 2^20].

At these sizes the oracle checks the output by the properties that single out the stable
sort under the index payload (permutation, key/payload agreement, order, ties in input
order; oracle.check_index_payload, O(n)), and by the rank formula evaluated one record at a
time for sampled output positions (oracle.rank_of, O(n) each).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

CASES = [(32, d, 1 << 28) for d in ("uniform", "normal", "zipf", "sorted", "reverse", "few")]
CASES += [(64, d, 1 << 27) for d in ("uniform", "skewed")]


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2207_14334_amd as dfr
    assert torch.cuda.is_available()
    ctx = dfr.Context(0)
    yield torch, dfr, ctx
    ctx.close()


@pytest.mark.parametrize("bits,dist,n", CASES, ids=[f"u{b}-{d}" for b, d, _ in CASES])
def test_full_size(env, bits, dist, n):
    torch, dfr, ctx = env
    o = oracle.get()
    print(f"[case] full-size u{bits} {dist} n={n}", flush=True)
    keys = workloads.make_keys(dist, n, bits, 0)
    vals = workloads.index_payload(n, bits)
    dk = torch.from_numpy(keys).cuda()
    dv = torch.from_numpy(vals).cuda()
    kb = bits // 8
    temp = torch.empty(dfr.temp_bytes(n, kb, kb), dtype=torch.uint8, device="cuda")
    ctx.sort_(dk, dv, temp)
    torch.cuda.synchronize()
    st = ctx.stats()
    del temp
    ok, ov = dk.cpu().numpy(), dv.cpu().numpy()
    del dk, dv
    assert o.check_index_payload(keys, ok, ov) is None, st
    rng = np.random.default_rng(n + bits)
    for p in rng.integers(0, n, size=3):
        assert o.rank_of(keys, int(ov[p])) == int(p), (dist, int(p))
    print(f"[done] {dist}: levels={st['levels']} top_digits={st['top_digits']} "
          f"deal_passes={st['deal_passes']} large={st['large_buckets']}", flush=True)


# Batched segmented sort at its full size: 20,000 uint32 arrays, lengths log-uniform
# in [16, 2^20] (about 1.9e9 keys in total), global index payload, uniform and Zipf keys.
@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_batched_full_size(env, dist):
    torch, dfr, ctx = env
    o = oracle.get()
    lens = workloads.batch_lengths(20000, 16, 1 << 20, 0)
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    print(f"[case] batched full-size {dist} arrays={lens.size} n={n}", flush=True)
    keys = workloads.make_keys(dist, n, 32, 0)
    vals = workloads.index_payload(n)
    dk = torch.from_numpy(keys).cuda()
    dv = torch.from_numpy(vals).cuda()
    ctx.sort_segmented_(dk, dv, off)
    torch.cuda.synchronize()
    st = ctx.stats()
    ok, ov = dk.cpu().numpy(), dv.cpu().numpy()
    del dk, dv
    torch.cuda.empty_cache()
    for s in range(lens.size):
        a, b = int(off[s]), int(off[s + 1])
        bad = o.check_index_payload(keys[a:b], ok[a:b], ov[a:b] - np.uint32(a))
        assert bad is None, (s, bad, st)
    rng = np.random.default_rng(7)
    for s in rng.integers(0, lens.size, size=3):
        a, b = int(off[s]), int(off[s + 1])
        p = int(rng.integers(a, b))
        assert o.rank_of(keys[a:b], int(ov[p]) - a) == p - a, (s, p)
    print(f"[done] batched {dist}: levels={st['levels']} deal_passes={st['deal_passes']}", flush=True)


# The size limit of the boundary.  The paper's largest input, 256^3.75 = 2^30 records
# (Fig. 1 and Fig. 2): uniform 32-bit keys with the uint32 index payload, checked by the
# same properties and sampled ranks as above.
@pytest.mark.timeout(900)
def test_paper_largest_size(env):
    torch, dfr, ctx = env
    o = oracle.get()
    n = 1 << 30
    print(f"[case] paper's largest size u32 uniform n={n}: generating", flush=True)
    keys = workloads.make_keys("uniform", n, 32, 5)
    vals = workloads.index_payload(n)
    dk = torch.from_numpy(keys).cuda()
    dv = torch.from_numpy(vals).cuda()
    del vals
    print(f"[case] n={n}: sorting", flush=True)
    ctx.sort_(dk, dv)
    torch.cuda.synchronize()
    st = ctx.stats()
    ok, ov = dk.cpu().numpy(), dv.cpu().numpy()
    del dk, dv
    torch.cuda.empty_cache()
    print(f"[case] n={n}: checking", flush=True)
    assert o.check_index_payload(keys, ok, ov) is None, st
    rng = np.random.default_rng(n)
    for p in rng.integers(0, n, size=2):
        assert o.rank_of(keys, int(ov[p])) == int(p), int(p)
    print(f"[done] n={n}: levels={st['levels']} deal_passes={st['deal_passes']}", flush=True)


# The most records one call accepts, 2^32 - 1: distinct keys k_i = (a i + b) mod 2^32
# (a odd), so the stable sort is the increasing order of the keys, which is every 32-bit
# value but the one that index n would have taken; the record holding value x came from
# index (x - b) / a mod 2^32.  The whole output is checked against that, chunk by chunk,
# and the rank formula at sampled places.
@pytest.mark.timeout(900)
def test_size_limit_records(env):
    torch, dfr, ctx = env
    o = oracle.get()
    n = dfr.MAX_SEGMENT_RECORDS
    assert n == (1 << 32) - 1
    print(f"[case] size limit n={n}: generating", flush=True)
    keys, a, b = workloads.permutation_keys(n, 9)
    dk = torch.from_numpy(keys).cuda()
    dv = torch.from_numpy(workloads.index_payload(n)).cuda()
    print(f"[case] n={n}: sorting", flush=True)
    ctx.sort_(dk, dv)
    torch.cuda.synchronize()
    st = ctx.stats()
    ok, ov = dk.cpu().numpy(), dv.cpu().numpy()
    del dk, dv
    torch.cuda.empty_cache()
    print(f"[case] n={n}: checking {st}", flush=True)
    mask = (1 << 32) - 1
    missing = (a * n + b) & mask
    a_inv = pow(a, -1, 1 << 32)
    step = 1 << 26
    for lo in range(0, n, step):
        p = np.arange(lo, min(n, lo + step), dtype=np.uint64)
        x = p + (p >= np.uint64(missing)).astype(np.uint64)
        src = ((x - np.uint64(b)) * np.uint64(a_inv)) & np.uint64(mask)
        assert np.array_equal(ok[lo:lo + p.size], x.astype(np.uint32)), lo
        assert np.array_equal(ov[lo:lo + p.size], src.astype(np.uint32)), lo
    rng = np.random.default_rng(3)
    for q in rng.integers(0, n, size=2):
        assert o.rank_of(keys, int(ov[q])) == int(q), int(q)
    print(f"[done] n={n}: levels={st['levels']} deal_passes={st['deal_passes']}", flush=True)


# The headline shape dealt the Fast Radix way (estimated buckets for the first deal).
@pytest.mark.parametrize("bits,n", [(32, 1 << 28), (64, 1 << 27)], ids=["u32-2p28", "u64-2p27"])
def test_full_size_estimated_buckets(env, bits, n):
    torch, dfr, ctx = env
    o = oracle.get()
    print(f"[case] full-size estimated buckets u{bits} n={n}", flush=True)
    keys = workloads.make_keys("uniform", n, bits, 0)
    vals = workloads.index_payload(n, bits)
    dk = torch.from_numpy(keys).cuda()
    dv = torch.from_numpy(vals).cuda()
    ctx.set_option("estimated_buckets", 1)
    try:
        ctx.sort_(dk, dv)
        torch.cuda.synchronize()
        st = ctx.stats()
    finally:
        ctx.set_option("estimated_buckets", 0)
    ok, ov = dk.cpu().numpy(), dv.cpu().numpy()
    del dk, dv
    assert st["deal_passes_estimated"] == 1, st
    assert o.check_index_payload(keys, ok, ov) is None, st
    rng = np.random.default_rng(n + 1)
    for p in rng.integers(0, n, size=2):
        assert o.rank_of(keys, int(ov[p])) == int(p), int(p)
