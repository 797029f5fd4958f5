"""GPU parity: the HIP path against the CPU oracle, element by element.

Every result here is integer work with a unique answer (the stable sort), so parity is
bit-exact.  Each test prints the case it is about to run before the GPU call.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2207_14334_amd as dfr
    c = dfr.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def o():
    return oracle.get()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def gpu_sort(torch, ctx, keys, vals, **opts):
    for k, v in opts.items():
        ctx.set_option(k, v)
    try:
        dk = dev(torch, keys)
        dv = dev(torch, vals) if vals is not None else None
        ctx.sort_(dk, dv)
        torch.cuda.synchronize()
        return host(dk), (host(dv) if dv is not None else None), ctx.stats()
    finally:
        for k in opts:
            ctx.set_option(k, 0)


def load_golden(name):
    d = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split(":", 1)
        d[k.strip()] = [int(x) for x in v.split()]
    return d


# --------------------------------------------------------------------------------------
# Stages: count and deal (Sec. 2).
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["counting_sort_0_9.txt", "cards_lsd.txt"])
def test_golden_count_deal(torch, ctx, name):
    g = load_golden(name)
    say("golden", name)
    k = np.array(g["keys"], dtype=np.uint32)
    v = np.array(g["vals"], dtype=np.uint32)
    h = host(ctx.count(dev(torch, k), bits=g["bits"][0], num_digits=1))
    assert list(h[0][:16]) == g["count"]
    dk, dv = ctx.deal(dev(torch, k), dev(torch, v), shift=g["shift"][0], bits=g["bits"][0])
    assert list(host(dk)) == g["deal_keys"] and list(host(dv)) == g["deal_vals"]
    sk, sv, _ = gpu_sort(torch, ctx, k, v)
    assert list(sk) == g["sorted_keys"] and list(sv) == g["sorted_vals"]


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal"])
def test_count_matches_oracle(torch, ctx, o, kb, dist):
    n = (1 << 20) + 12345
    k = workloads.make_keys(dist, n, 8 * kb, 3)
    say("count", dist, kb, n)
    h = host(ctx.count(dev(torch, k)))
    for j in range(kb):
        assert np.array_equal(h[j].astype(np.uint64), o.count(k, 8 * j, 8)), j


@pytest.mark.parametrize("kb,vb", [(4, 0), (4, 4), (8, 8), (8, 0)])
@pytest.mark.parametrize("shift,bits", [(0, 8), (8, 8), (3, 5), (24, 8), (0, 1)])
def test_deal_matches_oracle(torch, ctx, o, kb, vb, shift, bits):
    n = 3 * 8192 + 777  # several tiles and a ragged tail
    k = workloads.make_keys("zipf", n, 8 * kb, shift + bits)
    v = workloads.index_payload(n, 8 * vb) if vb else None
    say("deal", kb, vb, shift, bits, n)
    dk, dv = ctx.deal(dev(torch, k), dev(torch, v) if vb else None, shift=shift, bits=bits)
    rk, rv = o.deal(k, v, shift, bits)
    assert np.array_equal(host(dk), rk)
    if vb:
        assert np.array_equal(host(dv), rv)


# --------------------------------------------------------------------------------------
# Whole sort against the oracle.
# --------------------------------------------------------------------------------------

SIZES = [0, 1, 2, 3, 63, 64, 65, 1000, 4095, 4096, 4097, 8191, 8192, 8193, 20000, 65543,
         (1 << 20) + 3]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kb,vb", [(4, 4), (8, 8), (4, 0)])
def test_sort_sizes(torch, ctx, o, n, kb, vb):
    k = workloads.make_keys("uniform", n, 8 * kb, n)
    v = workloads.index_payload(n, 8 * vb) if vb else None
    say("sort", n, kb, vb)
    sk, sv, _ = gpu_sort(torch, ctx, k, v)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk)
    if vb:
        assert np.array_equal(sv, rv)


DISTS32 = ["uniform", "normal", "zipf", "sorted", "reverse", "few", "equal", "narrow"]


@pytest.mark.parametrize("dist", DISTS32)
@pytest.mark.parametrize("n", [1 << 18, (1 << 22) + 5])
def test_sort_distributions_u32(torch, ctx, o, dist, n):
    k = workloads.make_keys(dist, n, 32, 1)
    v = workloads.index_payload(n)
    say("sort32", dist, n)
    sk, sv, st = gpu_sort(torch, ctx, k, v)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st


@pytest.mark.parametrize("dist", ["uniform", "skewed", "normal", "zipf", "few", "equal"])
def test_sort_distributions_u64(torch, ctx, o, dist):
    n = (1 << 21) + 17
    k = workloads.make_keys(dist, n, 64, 2)
    v = workloads.index_payload(n, 64)
    say("sort64", dist, n)
    sk, sv, st = gpu_sort(torch, ctx, k, v)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("dist", ["uniform", "normal", "few"])
def test_forced_top_digits(torch, ctx, o, d, dist):
    """Every choice of d gives the same result; small d forces recursion on large buckets."""
    n = (1 << 21) + 99
    k = workloads.make_keys(dist, n, 32, d)
    v = workloads.index_payload(n)
    say("force_d", d, dist, n)
    sk, sv, st = gpu_sort(torch, ctx, k, v, force_top_digits=d)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    if d == 1 and dist == "uniform":
        assert st["levels"] >= 2 and st["large_buckets"] > 0, st


@pytest.mark.parametrize("divert", [16, 512, 8192])
def test_divert_threshold(torch, ctx, o, divert):
    n = (1 << 21) + 1
    k = workloads.make_keys("uniform", n, 32, 5)
    v = workloads.index_payload(n)
    say("divert", divert)
    sk, sv, st = gpu_sort(torch, ctx, k, v, divert_records=divert)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st


def test_deterministic_repeats(torch, ctx, o):
    n = (1 << 22) + 11
    k = workloads.make_keys("few", n, 32, 9)
    v = workloads.index_payload(n)
    say("repeat", n)
    first = None
    for _ in range(5):
        sk, sv, _ = gpu_sort(torch, ctx, k, v)
        if first is None:
            first = (sk, sv)
        assert np.array_equal(sk, first[0]) and np.array_equal(sv, first[1])
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(first[0], rk) and np.array_equal(first[1], rv)


# --------------------------------------------------------------------------------------
# Segmented sort.
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("dist", ["uniform", "zipf"])
@pytest.mark.parametrize("kb", [4, 8])
def test_segmented(torch, ctx, o, dist, kb):
    lens = workloads.batch_lengths(400, 1, 40000, 7)
    lens[3] = 0
    lens[10] = 1
    lens[11] = 9000
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    k = workloads.make_keys(dist, n, 8 * kb, 4)
    v = workloads.index_payload(n, 8 * kb)
    say("segmented", dist, kb, n, lens.size)
    dk, dv = dev(torch, k), dev(torch, v)
    ctx.sort_segmented_(dk, dv, off)
    torch.cuda.synchronize()
    rk, rv = o.segmented_sort(k, v, off)
    assert np.array_equal(host(dk), rk) and np.array_equal(host(dv), rv)


# --------------------------------------------------------------------------------------
# Argument errors leave the buffers untouched.
# --------------------------------------------------------------------------------------

def test_argument_errors(torch, ctx):
    import paper_2207_14334_amd as dfr
    k = dev(torch, np.arange(100, 0, -1, dtype=np.uint32))
    small = torch.empty(10, dtype=torch.uint8, device="cuda")
    with pytest.raises(dfr.DfrError) as e:
        ctx.sort_(k, None, temp=small)
    assert e.value.status == dfr.E_INVALID_ARG
    assert host(k)[0] == 100
    with pytest.raises(dfr.DfrError) as e:
        ctx.sort_(k, k)  # keys and vals overlap
    assert e.value.status == dfr.E_INVALID_ARG
    with pytest.raises(dfr.DfrError) as e:
        ctx.set_option("no_such_option", 1)
    assert e.value.status == dfr.E_UNSUPPORTED


def test_repeat_stress_many_tiles(torch, ctx, o):
    """Repeated large sorts must agree bit for bit (a race in a kernel shows up as a
    difference between repeats) and match the oracle."""
    for dist, n in (("uniform", (1 << 24) + 77), ("normal", 1 << 23)):
        k = workloads.make_keys(dist, n, 32, 21)
        v = workloads.index_payload(n)
        say("stress", dist, n)
        first = None
        for _ in range(6):
            sk, sv, _ = gpu_sort(torch, ctx, k, v)
            if first is None:
                first = (sk, sv)
            assert np.array_equal(sk, first[0]) and np.array_equal(sv, first[1]), dist
        assert o.check_index_payload(k, first[0], first[1]) is None, dist


# --------------------------------------------------------------------------------------
# Both ways of finding a tile's place in its buckets: scanned ahead of the deal from
# per-tile counts, or decoupled look-back between tiles.  Same result either way.
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("lookback", [0, 1])
@pytest.mark.parametrize("case", ["single", "recursion", "segmented", "long_segment"])
def test_deal_modes(torch, ctx, o, case, lookback):
    kb = 4
    opts = {"force_lookback": lookback}
    if case == "single":
        n = (1 << 21) + 333
        off = None
    elif case == "recursion":
        n = (1 << 22) + 5
        off = None
        opts["force_top_digits"] = 1  # 256 large buckets: a multi-segment second level
    elif case == "segmented":
        lens = workloads.batch_lengths(300, 1, 1 << 18, 12)
        off = workloads.segment_offsets(lens)
        n = int(off[-1])
    else:
        # One segment over more tiles than a single block scans ahead, among more
        # segments than are scanned one by one: the level falls back to look-back
        # between tiles even with the option off.
        lens = np.array([5, (1 << 23) + 8192 * 3 + 11, 70000, 0, 9000] + [12000] * 20,
                        dtype=np.int64)
        off = workloads.segment_offsets(lens)
        n = int(off[-1])
    k = workloads.make_keys("uniform", n, 8 * kb, 31)
    v = workloads.index_payload(n)
    say("deal_modes", case, lookback, n)
    for name, val in opts.items():
        ctx.set_option(name, val)
    try:
        dk, dv = dev(torch, k), dev(torch, v)
        if off is None:
            ctx.sort_(dk, dv)
        else:
            ctx.sort_segmented_(dk, dv, off)
        torch.cuda.synchronize()
        st = ctx.stats()
    finally:
        for name in opts:
            ctx.set_option(name, 0)
    if off is None:
        rk, rv = o.stable_sort(k, v)
    else:
        rk, rv = o.segmented_sort(k, v, off)
    assert np.array_equal(host(dk), rk) and np.array_equal(host(dv), rv), st
    # The intended deal form ran.
    assert st["deal_passes"] == st["deal_passes_scanned"] + st["deal_passes_lookback"], st
    if lookback or case == "long_segment":
        assert st["deal_passes_lookback"] > 0, st
    else:
        assert st["deal_passes_lookback"] == 0 and st["deal_passes_scanned"] > 0, st


@pytest.mark.parametrize("bits", [32, 64])
def test_segmented_mixed_plans(torch, ctx, o, bits):
    """Segments of different distributions get different digit plans in one level
    (full LSD for some, one or two top digits for others, passes sat out in pairs
    and an odd leftover dealt twice); every segment must still match the oracle."""
    parts = [("zipf", 300000), ("uniform", 300000), ("few", 200000), ("narrow", 100000),
             ("equal", 50000), ("sorted", 250000), ("uniform", 20000), ("normal", 9000),
             ("zipf", 9000), ("reverse", 70000)]
    if bits == 64:
        parts.append(("skewed", 200000))
    keys = [workloads.make_keys(dname, m, bits, 40 + i) for i, (dname, m) in enumerate(parts)]
    lens = np.array([m for _, m in parts], dtype=np.int64)
    off = workloads.segment_offsets(lens)
    k = np.concatenate(keys)
    n = k.size
    v = workloads.index_payload(n, bits)
    rk, rv = o.segmented_sort(k, v, off)
    # Plans from each segment's digit histograms (the read-back plan, the default), and
    # from the lengths alone.
    for from_hist in (1, 0):
        say("segmented_mixed", bits, n, "histogram plans" if from_hist else "length plans")
        if not from_hist:
            ctx.set_option("plan_lengths_records", 1 << 22)
        try:
            dk, dv = dev(torch, k), dev(torch, v)
            ctx.sort_segmented_(dk, dv, off)
            torch.cuda.synchronize()
            st = ctx.stats()
        finally:
            ctx.set_option("plan_lengths_records", 0)
        assert np.array_equal(host(dk), rk) and np.array_equal(host(dv), rv), st
        assert st["plan_from_lengths"] == 1 - from_hist, st


@pytest.mark.parametrize("dist", ["uniform", "zipf", "few", "narrow", "equal", "sorted"])
def test_plan_from_lengths(torch, ctx, o, dist):
    """With the plan_lengths_records option, a first level of short segments picks its
    top digits from its length alone (no read-back before its deals): skewed, narrow or
    constant keys then leave large buckets for the next level or deal digits that do not
    vary; the result matches the oracle either way, and the same as the histogram plan."""
    n = (1 << 21) + 77
    k = workloads.make_keys(dist, n, 32, 19)
    v = workloads.index_payload(n)
    say("plan from lengths", dist, n)
    sk, sv, st = gpu_sort(torch, ctx, k, v, plan_lengths_records=1 << 22)
    hk, hv, ht = gpu_sort(torch, ctx, k, v)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    assert np.array_equal(hk, rk) and np.array_equal(hv, rv), ht
    assert st["plan_from_lengths"] == 1 and st["top_digits"] == 2, st
    assert ht["plan_from_lengths"] == 0, ht


@pytest.mark.parametrize("bits,n", [(32, (1 << 25) + 12345), (64, (1 << 23) + 77)])
def test_skewed_prefix_recursion(torch, ctx, o, bits, n):
    """The top digit takes 4 values: the level deals it alone and each of the 4 large
    buckets is planned on its own (the 32-bit case puts more than 1024 tiles in each
    bucket, so the next level scans each bucket's tiles with the one-segment scan)."""
    rng = np.random.default_rng(bits)
    dt = np.uint32 if bits == 32 else np.uint64
    low_bits = bits - 8
    top = rng.choice(256, size=4, replace=False).astype(dt)
    low = workloads.make_keys("uniform", n, bits, 77) & dt((1 << low_bits) - 1)
    k = (top[rng.integers(0, 4, n)] << dt(low_bits)) | low
    v = workloads.index_payload(n, bits)
    say("skewed prefix", bits, n)
    sk, sv, st = gpu_sort(torch, ctx, k, v)
    assert st["levels"] >= 2 and st["top_digits"] == 1, st
    assert o.check_index_payload(k, sk, sv) is None, st
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st


@pytest.mark.parametrize("dist", ["uniform", "zipf", "normal"])
def test_estimated_overflow(torch, ctx, o, dist):
    """The overflow Fast Radix's estimated buckets would meet on the top varying digit
    (Sec. 3.1): exactly the count the histogram gives, and for uniform keys close to the
    expectation of Eq. 2."""
    n = 1 << 24
    k = workloads.make_keys(dist, n, 32, 8)
    say("estimated overflow", dist, n)
    _, _, st = gpu_sort(torch, ctx, k, None)
    orv = np.bitwise_or.reduce(k) ^ np.bitwise_and.reduce(k)
    top = max(j for j in range(4) if (int(orv) >> (8 * j)) & 0xFF)
    h = np.bincount(((k >> np.uint32(8 * top)) & np.uint32(0xFF)).astype(np.int64), minlength=256)
    cap = -(-n // 256)
    expect = float(np.maximum(h - cap, 0).sum()) / float(n)
    assert st["estimated_overflow"] == expect, (st["estimated_overflow"], expect)
    if dist == "uniform":
        eq2 = o.overflow_fraction(n, 256)
        assert abs(st["estimated_overflow"] / eq2 - 1) < 0.25, (st["estimated_overflow"], eq2)


def test_segmented_device_offsets(torch, ctx, o):
    """Offsets may live in device memory; the result is the same."""
    lens = workloads.batch_lengths(200, 1, 30000, 9)
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    k = workloads.make_keys("uniform", n, 32, 9)
    v = workloads.index_payload(n)
    say("segmented device offsets", n)
    dk, dv = dev(torch, k), dev(torch, v)
    doff = torch.from_numpy(off.astype(np.int64)).cuda()
    ctx.sort_segmented_(dk, dv, doff)
    torch.cuda.synchronize()
    rk, rv = o.segmented_sort(k, v, off)
    assert np.array_equal(host(dk), rk) and np.array_equal(host(dv), rv)


# --------------------------------------------------------------------------------------
# Edge cases of the key range and of the local sort's capacity.
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("n", [3, 4097, (1 << 20) + 3])
def test_keys_only_extremes(torch, ctx, o, bits, n):
    dt = np.uint32 if bits == 32 else np.uint64
    rng = np.random.default_rng(n)
    k = np.where(rng.integers(0, 2, n) == 1, np.iinfo(dt).max, 0).astype(dt)
    v = workloads.index_payload(n, bits)
    say("extremes", bits, n)
    sk, sv, st = gpu_sort(torch, ctx, k, v)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st


@pytest.mark.parametrize("kb", [4, 8])
def test_buckets_at_capacity(torch, ctx, o, kb):
    """Top-digit buckets of exactly the local sort's capacity C, of C + 1 (then sorted by
    the next level), of C - 1, and of one record."""
    import paper_2207_14334_amd as dfr
    cap = dfr.local_sort_capacity(kb, kb)
    sizes = [cap, cap + 1, cap - 1, 1, cap, 2 * cap + 1]
    bits = 8 * kb
    dt = np.uint32 if kb == 4 else np.uint64
    parts = []
    for b, m in enumerate(sizes):
        low = workloads.make_keys("uniform", m, bits, 100 + b) >> dt(8)
        parts.append((dt(37 * b + 5) << dt(bits - 8)) | low)
    k = np.concatenate(parts)
    rng = np.random.default_rng(kb)
    k = k[rng.permutation(k.size)]
    v = workloads.index_payload(k.size, bits)
    say("buckets at capacity", kb, k.size)
    sk, sv, st = gpu_sort(torch, ctx, k, v, force_top_digits=1, divert_records=cap)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    # Buckets of C records exceed the bucketed kernels' chunk: the general kernel sorts
    # them; C + 1 and 2C + 1 recurse.
    assert st["chunks_general"] >= 2 and st["levels"] >= 2, st


FORM_CASES = [
    # (key bits, payload bits, n, segmented, form expected): the headline shape (two
    # digits of 32-bit keys dealt, buckets of ~1024 records or more: 32-bit words with
    # the position inside); one digit of 32-bit keys dealt (position beside the words);
    # two digits dealt into buckets of ~64 records, about 32 to a window, whose index
    # leaves no room for the position (beside the words from the start); 64-bit keys
    # with buckets of ~256 records or more (64-bit words).
    (32, 32, (1 << 26) + 7, False, 0),
    (32, 32, (1 << 20) + 3, False, 1),
    (32, 32, (1 << 22) + 3, False, 1),
    (32, 32, None, True, 1),
    (64, 64, (1 << 24) + 5, False, 2),
    (32, 0, (1 << 26) + 1, False, 0),
]


@pytest.mark.parametrize("bits,vbits,n,segmented,form", FORM_CASES,
                         ids=[f"u{b}v{vb}-{n}-{'seg' if g else 'plain'}-form{f}"
                              for b, vb, n, g, f in FORM_CASES])
def test_local_sort_forms(torch, ctx, o, bits, vbits, n, segmented, form):
    """Each form of the bucketed local sort is the one that runs for its shape, and
    the result matches the oracle."""
    if segmented:
        lens = workloads.batch_lengths(200, 16, 1 << 17, 21)
        off = workloads.segment_offsets(lens)
        n = int(off[-1])
    k = workloads.make_keys("uniform", n, bits, 61)
    v = workloads.index_payload(n, vbits) if vbits else None
    say("local sort forms", bits, vbits, n, segmented, form)
    dk = dev(torch, k)
    dv = dev(torch, v) if v is not None else None
    if segmented:
        ctx.sort_segmented_(dk, dv, off)
    else:
        ctx.sort_(dk, dv)
    torch.cuda.synchronize()
    st = ctx.stats()
    if segmented:
        rk, rv = o.segmented_sort(k, v, off)
        assert np.array_equal(host(dk), rk) and np.array_equal(host(dv), rv), st
    elif n > 1 << 24 and v is not None:  # the stable sort's properties, sampled ranks
        sk, sv = host(dk), host(dv)
        assert o.check_index_payload(k, sk, sv) is None, st
        for p in np.random.default_rng(n).integers(0, n, size=2):
            assert o.rank_of(k, int(sv[p])) == int(p), int(p)
    elif n > 1 << 24:  # keys only: the sorted multiset (numpy, an independent library)
        assert np.array_equal(host(dk), np.sort(k)), st
    else:
        rk, rv = o.stable_sort(k, v)
        assert np.array_equal(host(dk), rk), st
        if v is not None:
            assert np.array_equal(host(dv), rv), st
    forms = [st["chunks_form0"], st["chunks_form1"], st["chunks_form2"]]
    assert forms[form] > 0, st
    if form < 2:  # the other 32-bit form is never chosen for the same level
        assert forms[1 - form] == 0, st
    # Every work item is sorted by exactly one kernel (hand-offs count where they end).
    assert sum(forms) + st["chunks_general"] == st["chunks"], st


def test_local_sort_hand_on_to_wide_form(torch, ctx, o):
    """Two top digits of 2^24 32-bit keys average 256 records a bucket, about 8 to a
    window of 2048, so the level starts with form 0 (16 varying bits, 3 of bucket index
    and a 13-bit position fill 32 bits).  Here 7/8 of the records fall in the lower half
    of the top-16-bit values (buckets of ~448) and 1/8 in the upper half (buckets of
    ~64): a window there holds about 32 buckets, too many for form 0, which hands those
    chunks' descriptors on to the 64-bit form (the diversion of Sec. 3)."""
    n = (1 << 24) - 3
    rng = np.random.default_rng(71)
    hot = rng.random(n) < 7 / 8
    top = np.where(hot, rng.integers(0, 1 << 15, n), rng.integers(1 << 15, 1 << 16, n)).astype(np.uint32)
    k = (top << np.uint32(16)) | (workloads.make_keys("uniform", n, 32, 71) >> np.uint32(16))
    v = workloads.index_payload(n, 32)
    say("hand on to the 64-bit form", n)
    sk, sv, st = gpu_sort(torch, ctx, k, v, force_top_digits=2)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    assert st["levels"] == 1 and st["chunks_form1"] == 0, st
    assert st["chunks_form0"] > 0 and st["chunks_form2"] > 0, st
    assert st["chunks_form0"] + st["chunks_form2"] + st["chunks_general"] == st["chunks"], st


def test_local_sort_hand_on_to_general(torch, ctx, o):
    """Buckets of about 4096 records whose 16 low bits vary only in bit 15 and bits 0-3:
    binned by the top 12 of those bits, each bucket falls into two bins of about 2048
    records, far above the 64 the bucketed form ranks, so its descriptor is handed on to
    the stable LSD kernel, which sorts it."""
    n = (1 << 20) + 5
    rng = np.random.default_rng(73)
    top = rng.integers(0, 256, n).astype(np.uint32) << np.uint32(24)
    mid = np.uint32(0x5a) << np.uint32(16)
    low = (rng.integers(0, 2, n).astype(np.uint32) << np.uint32(15)) | rng.integers(0, 16, n).astype(np.uint32)
    k = top | mid | low
    v = workloads.index_payload(n, 32)
    say("hand on to the general kernel", n)
    sk, sv, st = gpu_sort(torch, ctx, k, v, force_top_digits=2)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    assert st["levels"] == 1 and st["chunks_general"] > 0, st
    assert sum(st[f"chunks_form{i}"] for i in range(3)) + st["chunks_general"] == st["chunks"], st


@pytest.mark.parametrize("spacing", [1, 2, 3, 4, 16])
@pytest.mark.parametrize("kb", [4, 8])
def test_local_sort_bucket_spacing(torch, ctx, o, spacing, kb):
    """Runs of small buckets whose top-16-bit values are spaced 1, 2, 3, 4 or 16 apart:
    the local sort takes a bucket's index from the key itself while the chunk's buckets
    span at most about twice as many values as there are buckets, and from the bucket
    starts otherwise; both rebuild the bits above the sorted ones."""
    bits = 8 * kb
    dt = np.uint32 if kb == 4 else np.uint64
    n = (1 << 20) + 7
    rng = np.random.default_rng(1000 * kb + spacing)
    top = (rng.integers(0, 4096, n) * spacing + 5).astype(dt)
    low = workloads.make_keys("uniform", n, bits, spacing) >> dt(16)
    k = (top << dt(bits - 16)) | low
    v = workloads.index_payload(n, bits)
    say("bucket spacing", spacing, kb, n)
    sk, sv, st = gpu_sort(torch, ctx, k, v, force_top_digits=2)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    assert st["levels"] == 1, st


HEADS_CASES = [
    # (key bits, n, distribution, radix bits, forced top digits)
    (32, 5, "uniform", 0, 2),
    (32, 8191, "uniform", 0, 2),
    (32, 8193, "uniform", 0, 2),
    (32, (1 << 20) + 3, "uniform", 0, 2),
    (32, (1 << 22) + 9, "uniform", 0, 0),
    (32, (1 << 21) + 1, "normal", 0, 2),
    (32, (1 << 21) + 1, "few", 0, 2),
    (32, (1 << 21) + 1, "narrow", 0, 2),
    (32, (1 << 20) + 11, "uniform", 6, 2),
    (32, (1 << 20) + 11, "uniform", 7, 2),
    (64, (1 << 20) + 5, "uniform", 0, 2),
    (64, (1 << 20) + 5, "skewed", 0, 2),
    (32, (1 << 21) + 1, "uniform", 0, 1),
    (32, 70001, "uniform", 0, 1),
    (64, (1 << 20) + 5, "skewed", 0, 0),
]


@pytest.mark.parametrize("bits,n,dist,rb,d", HEADS_CASES,
                         ids=[f"u{b}-{n}-{t}-rb{r}-d{d}" for b, n, t, r, d in HEADS_CASES])
def test_heads_from_counts(torch, ctx, o, bits, n, dist, rb, d):
    """A one-segment level dealt on two digits lists its buckets from the digit counts
    (first digit's histogram, second deal's per-tile counts, and the keys of the tiles
    that straddle a first-digit range), one dealt on one digit from its histogram; the
    same sort with the heads found from the keys gives the same chunks and the same,
    stable result."""
    k = workloads.make_keys(dist, n, bits, 77)
    v = workloads.index_payload(n, bits)
    opts = {"force_top_digits": d}
    if rb:
        opts["radix_bits"] = rb
    say("heads from counts", bits, n, dist, rb, d)
    sk, sv, st = gpu_sort(torch, ctx, k, v, **opts)
    say("heads from keys", bits, n, dist, rb, d)
    fk, fv, ft = gpu_sort(torch, ctx, k, v, force_key_heads=1, **opts)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    assert np.array_equal(fk, rk) and np.array_equal(fv, rv), ft
    assert st["chunks"] == ft["chunks"] and st["levels"] == ft["levels"], (st, ft)
    # The forced run found every level's heads from the keys.
    assert ft["levels_heads_counts"] == 0 and ft["levels_heads_hist"] == 0, ft
    if st["used_diversion"] and n > 8192:
        assert ft["levels_heads_keys"] >= 1, ft
    # The unforced run took the counts (two digits dealt) or histograms (one digit) on
    # its first level when the plan allowed it.
    if st["top_digits"] == 2 and st["used_diversion"] and n > 8192 and not rb:
        assert st["levels_heads_counts"] >= 1, st
    if st["top_digits"] == 1 and st["used_diversion"] and n > 8192:
        assert st["levels_heads_hist"] >= 1, st


@pytest.mark.parametrize("n,dist", [((1 << 25) + 77, "uniform"), ((1 << 26) + 3, "normal")])
def test_wide_default_windows(torch, ctx, o, n, dist):
    """Levels whose buckets average 512 records or more take windows of half the bucketed
    local sort's capacity by default; checked by the properties that single out the
    stable sort under the index payload, and the rank formula at sampled places."""
    k = workloads.make_keys(dist, n, 32, 91)
    v = workloads.index_payload(n)
    say("wide default windows", n, dist)
    sk, sv, st = gpu_sort(torch, ctx, k, v)
    assert o.check_index_payload(k, sk, sv) is None, st
    rng = np.random.default_rng(n)
    for p in rng.integers(0, n, size=3):
        assert o.rank_of(k, int(sv[p])) == int(p), (dist, int(p))


@pytest.mark.parametrize("kb,dist", [(4, "uniform"), (4, "normal"), (8, "uniform"), (4, "few")])
def test_segmented_heads_from_histograms(torch, ctx, o, kb, dist):
    """A segmented level dealt on one digit lists each segment's buckets from its digit
    histogram; the same sort with the heads found from the keys gives the same chunks
    and the same, stable result, per segment."""
    lens = workloads.batch_lengths(300, 16, 1 << 18, 11)
    lens[5] = 0
    lens[6] = 8193
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    k = workloads.make_keys(dist, n, 8 * kb, 12)
    v = workloads.index_payload(n, 8 * kb)
    out = []
    for force in (0, 1):
        say("segmented heads", kb, dist, n, "from keys" if force else "from histograms")
        ctx.set_option("force_key_heads", force)
        try:
            dk, dv = dev(torch, k), dev(torch, v)
            ctx.sort_segmented_(dk, dv, off)
            torch.cuda.synchronize()
            out.append((host(dk), host(dv), ctx.stats()))
        finally:
            ctx.set_option("force_key_heads", 0)
    rk, rv = o.segmented_sort(k, v, off)
    for sk, sv, st in out:
        assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    assert out[0][2]["chunks"] == out[1][2]["chunks"], (out[0][2], out[1][2])


def test_size_limit(torch, ctx):
    """More records than one segment may hold: refused before any work."""
    import ctypes
    import paper_2207_14334_amd as dfr
    k = dev(torch, np.arange(16, dtype=np.uint32))
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert dfr.MAX_SEGMENT_RECORDS == (1 << 32) - 1
    st = dfr.lib().dfr_sort_u32(ctx._h, k.data_ptr(), None, dfr.MAX_SEGMENT_RECORDS + 1, None, 0, s)
    assert st == dfr.E_TOO_LARGE
    # The same limit per segment of a segmented sort, and per serving request.
    off = np.array([0, 3, 3 + (1 << 32)], dtype=np.uint64)
    st = dfr.lib().dfr_sort_segmented_u32(ctx._h, k.data_ptr(), None, off.ctypes.data, 2, None, 0, s)
    assert st == dfr.E_TOO_LARGE
    with pytest.raises(dfr.DfrError) as e:
        r = dfr.Request(4, 0, k.data_ptr(), None, 1 << 32)
        t = ctypes.c_uint64(0)
        ctx._raise(dfr.lib().dfr_submit(ctx._h, ctypes.byref(r), ctypes.byref(t)), "submit")
    assert e.value.status == dfr.E_TOO_LARGE
    # A misaligned key pointer.
    assert dfr.lib().dfr_sort_u64(ctx._h, k.data_ptr() + 4, None, 2, None, 0, s) == dfr.E_INVALID_ARG
    assert np.array_equal(host(k), np.arange(16, dtype=np.uint32))


def test_lookback_determinism(torch, ctx, o):
    """Decoupled look-back with half tiles (longer chains) over a grid far larger than
    the resident blocks: repeats agree bit for bit and match the oracle."""
    import paper_2207_14334_amd as dfr
    n = (1 << 24) + 321
    k = workloads.make_keys("uniform", n, 32, 44)
    v = workloads.index_payload(n)
    say("lookback determinism", n)
    first = None
    for _ in range(4):
        sk, sv, _ = gpu_sort(torch, ctx, k, v, force_lookback=1,
                             tile_records=dfr.deal_tile_records(4, 4) // 2)
        if first is None:
            first = (sk, sv)
        assert np.array_equal(sk, first[0]) and np.array_equal(sv, first[1])
    assert o.check_index_payload(k, first[0], first[1]) is None


def test_calls_on_different_streams(torch, ctx, o):
    """Consecutive calls on one context from different streams, with no host wait
    between them: a 256-distinct-value sort (its last buckets copied back from the temp
    buffer after the call's last read-back) on stream A, then sorts on stream B that
    reuse the same scratch and temp buffer; every result matches the oracle."""
    n = (1 << 22) + 17
    ka = workloads.make_keys("few", n, 32, 71)
    kb = workloads.make_keys("uniform", n, 32, 72)
    v = workloads.index_payload(n)
    ra, rb = o.stable_sort(ka, v), o.stable_sort(kb, v)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        say("streams in turn", rep)
        da, dva, db, dvb = dev(torch, ka), dev(torch, v), dev(torch, kb), dev(torch, v)
        torch.cuda.synchronize()
        ctx.sort_(da, dva, stream=sa)
        ctx.sort_(db, dvb, stream=sb)
        ctx.sort_(dva, None, stream=sa)  # a third call back on A, on A's first result
        sa.synchronize()
        sb.synchronize()
        assert np.array_equal(host(da), ra[0]), rep
        assert np.array_equal(host(dva), np.sort(ra[1])), rep
        assert np.array_equal(host(db), rb[0]) and np.array_equal(host(dvb), rb[1]), rep


# --------------------------------------------------------------------------------------
# Fast Radix's estimated buckets (Sec. 3; overflow, Sec. 3.1), the "estimated_buckets"
# option: the first deal without a count, into buckets of n / 2^b slots plus overflow
# slots; levels whose buckets outgrow their slots are dealt with counted buckets.
# --------------------------------------------------------------------------------------

def _overflowing_keys(n, seed):
    """Uniform 32-bit keys whose bits 16..23 take the value 7 about 400 times more than
    their share: bucket 7 of the estimated deal overflows its n / 256 slots."""
    k = workloads.make_keys("uniform", n, 32, seed)
    rng = np.random.default_rng(seed)
    pick = rng.choice(n, 400, replace=False)
    k[pick] = (k[pick] & np.uint32(0xFF00FFFF)) | np.uint32(7 << 16)
    return k


EST_CASES = [
    # (key bits, distribution, n, estimated deal expected to be used)
    (32, "uniform", (1 << 22) + 5, True),
    (32, "normal", 1 << 22, True),       # bits 16..23 of the normal keys are near uniform
    (32, "overflow", 1 << 22, True),     # one bucket well over its estimate, within slots
    (32, "zipf", 1 << 22, False),        # most keys share bits 16..23: counted instead
    (32, "few", (1 << 21) + 1, False),
    (64, "uniform", (1 << 21) + 3, True),
    (64, "skewed", 1 << 21, False),
]


@pytest.mark.parametrize("bits,dist,n,used", EST_CASES, ids=[f"u{b}-{d}-{n}" for b, d, n, _ in EST_CASES])
def test_estimated_buckets(torch, ctx, o, bits, dist, n, used):
    k = _overflowing_keys(n, 3) if dist == "overflow" else workloads.make_keys(dist, n, bits, 3)
    v = workloads.index_payload(n, bits)
    say("estimated buckets", bits, dist, n)
    sk, sv, st = gpu_sort(torch, ctx, k, v, estimated_buckets=1)
    rk, rv = o.stable_sort(k, v)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st
    assert st["deal_passes_estimated"] == (1 if used else 0), st
    if used:
        assert st["top_digits"] == 2 and st["deal_passes_lookback"] >= 1, st
        # The overflow the estimated deal met, against the counts of the dealt digit.
        shift = 8 * (bits // 8) - 16
        h = np.bincount(((k >> k.dtype.type(shift)) & k.dtype.type(255)).astype(np.int64), minlength=256)
        e = n // 256
        assert st["estimated_overflow"] == pytest.approx(np.maximum(h - e, 0).sum() / n, abs=1e-12), st
    if dist == "overflow":
        assert st["estimated_overflow"] * n >= 300, st
