"""GPU parity at the benchmark's full sizes, in the configuration bench.py times.

2^28 uint32 keys with a uint32 index payload on each key distribution of that workload
(uniform, normal, Zipf, sorted, reverse-sorted, 256 distinct values), and 2^27 uint64
keys with a uint64 index payload (uniform, and top-16-bits-from-4-values skewed).

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
