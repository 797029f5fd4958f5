"""Pins of the CPU oracle to things other than itself.

The oracle's result is the stable sort (Sec. 2.1 stability, Sec. 3 DFR).  These tests
check it against:

* brute force: the one permutation, found by exhaustive search, that orders the keys
  and keeps equal keys in input order (a characterisation, not a construction);
* numpy's stable argsort, an independent library;
* the special cases whose output is known in closed form;
* the hand-worked instances of Sec. 2 (counting sort, keys 0-9) and Sec. 2.1 (cards)
  under tests/golden/;
* the four properties that single out the stable sort under the index payload.

Each pin is a function of an ``Oracle`` so that ``test_planted_mistakes`` can run the
same pins on copies of the oracle built with a mistake planted in them and check that
some pin fails for every such copy.
"""
from __future__ import annotations

import itertools
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

U32_EXTREMES = [0, 1, 1 << 31, (1 << 32) - 1]
U64_EXTREMES = [0, 1, 1 << 63, (1 << 64) - 1]


def load_golden(name):
    d = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split(":", 1)
            d[k.strip()] = [int(x) for x in v.split()]
    return d


def brute_stable_permutation(keys):
    """All permutations p with keys[p] ascending and ties in input order."""
    n = len(keys)
    found = []
    for p in itertools.permutations(range(n)):
        ok = True
        for a, b in zip(p, p[1:]):
            if keys[a] > keys[b] or (keys[a] == keys[b] and a > b):
                ok = False
                break
        if ok:
            found.append(p)
    return found


# --------------------------------------------------------------------------------------
# Pins, as functions of an oracle build.
# --------------------------------------------------------------------------------------

def pin_bruteforce_small_alphabet(o, max_n=6):
    for n in range(0, max_n + 1):
        for keys in itertools.product((0, 1, 2), repeat=n):
            k = np.array(keys, dtype=np.uint32)
            sols = brute_stable_permutation(keys)
            assert len(sols) == 1
            ok, ov = o.stable_sort(k, np.arange(n, dtype=np.uint32))
            assert list(ov) == list(sols[0]), keys
            assert list(ok) == [keys[i] for i in sols[0]], keys


def pin_bruteforce_extremes(o, max_n=5):
    for dt, alphabet in ((np.uint32, U32_EXTREMES), (np.uint64, U64_EXTREMES)):
        for n in range(0, max_n + 1):
            for keys in itertools.product(alphabet, repeat=n):
                sols = brute_stable_permutation(keys)
                assert len(sols) == 1
                k = np.array(keys, dtype=dt)
                ok, ov = o.stable_sort(k, np.arange(n, dtype=np.uint64))
                assert list(ov) == list(sols[0]), (dt, keys)


def pin_numpy(o):
    for seed, (dist, bits, n) in enumerate([
        ("uniform", 32, 100_000), ("zipf", 32, 50_000), ("few", 32, 70_001),
        ("normal", 32, 65_537), ("uniform", 64, 40_000), ("skewed", 64, 30_000),
        ("narrow", 32, 10_000), ("narrow", 64, 10_000),
    ]):
        k = workloads.make_keys(dist, n, bits, seed)
        ok, ov = o.stable_sort(k, workloads.index_payload(n, bits))
        ref = np.argsort(k, kind="stable")
        assert np.array_equal(ov, ref.astype(ov.dtype)), dist
        assert np.array_equal(ok, k[ref]), dist


def pin_special_cases(o):
    rng = np.random.default_rng(7)
    # sorted input -> identity
    k = np.sort(rng.integers(0, 1 << 32, 5000, dtype=np.uint32))
    ok, ov = o.stable_sort(k, np.arange(k.size, dtype=np.uint32))
    assert np.array_equal(ov, np.arange(k.size)) and np.array_equal(ok, k)
    # reverse-sorted distinct keys -> reversal
    k = np.unique(rng.integers(0, 1 << 32, 5000, dtype=np.uint32))[::-1].copy()
    ok, ov = o.stable_sort(k, np.arange(k.size, dtype=np.uint32))
    assert np.array_equal(ov, np.arange(k.size)[::-1])
    # reverse-sorted with duplicates -> ties keep ascending input order
    k = np.array([5, 5, 4, 4, 4, 1, 0, 0], dtype=np.uint32)
    _, ov = o.stable_sort(k, np.arange(8, dtype=np.uint32))
    assert list(ov) == [6, 7, 5, 2, 3, 4, 0, 1]
    # all-equal -> identity
    k = np.full(3000, 0xDEADBEEF, dtype=np.uint32)
    ok, ov = o.stable_sort(k, np.arange(3000, dtype=np.uint32))
    assert np.array_equal(ov, np.arange(3000))
    # n = 0 and n = 1
    ok, ov = o.stable_sort(np.empty(0, np.uint32), np.empty(0, np.uint32))
    assert ok.size == 0 and ov.size == 0
    ok, ov = o.stable_sort(np.array([9], np.uint64), np.array([0], np.uint64))
    assert list(ok) == [9] and list(ov) == [0]
    # 256 distinct values -> run lengths equal the input histogram
    k = workloads.make_keys("few", 100_000, 32, 3)
    ok, _ = o.stable_sort(k, None)
    vals, counts = np.unique(k, return_counts=True)
    run_starts = np.flatnonzero(np.r_[True, ok[1:] != ok[:-1]])
    run_lens = np.diff(np.r_[run_starts, ok.size])
    assert np.array_equal(ok[run_starts], vals) and np.array_equal(run_lens, counts)


def pin_golden(o):
    for name in ("counting_sort_0_9.txt", "cards_lsd.txt"):
        g = load_golden(name)
        k = np.array(g["keys"], dtype=np.uint32)
        v = np.array(g["vals"], dtype=np.uint32)
        shift, bits = g["shift"][0], g["bits"][0]
        assert list(o.count(k, shift, bits)) == g["count"], name
        dk, dv = o.deal(k, v, shift, bits)
        assert list(dk) == g["deal_keys"] and list(dv) == g["deal_vals"], name
        assert list(np.cumsum(o.count(k, shift, bits))[: len(g["index_after"])]) == g["index_after"]
        for sk, sv in (o.stable_sort(k, v), o.lsd_sort(k, v, bits=4), o.dfr_sort(k, v, 4, 2)):
            assert list(sk) == g["sorted_keys"] and list(sv) == g["sorted_vals"], name


def pin_properties(o):
    for dist, bits in (("uniform", 32), ("zipf", 32), ("few", 32), ("skewed", 64), ("equal", 64)):
        k = workloads.make_keys(dist, 50_000, bits, 11)
        ok, ov = o.stable_sort(k, workloads.index_payload(k.size, bits))
        assert o.check_index_payload(k, ok, ov) is None, dist


def pin_rank_formula(o):
    """The O(n^2) rank formula against brute force and numpy (not against the sort)."""
    for keys in itertools.product((0, 1, 2), repeat=5):
        sol = brute_stable_permutation(keys)[0]
        r = o.rank(np.array(keys, dtype=np.uint32))
        inv = np.empty(5, dtype=np.int64)
        inv[list(sol)] = np.arange(5)
        assert list(r) == list(inv), keys
    k = workloads.make_keys("few", 3000, 32, 5) >> np.uint32(26)
    r = o.rank(k)
    inv = np.empty(k.size, dtype=np.int64)
    inv[np.argsort(k, kind="stable")] = np.arange(k.size)
    assert np.array_equal(r, inv)
    for i in (0, 17, 2999):
        assert o.rank_of(k, i) == inv[i]


def load_typed_golden():
    d = {}
    for line in open(os.path.join(GOLDEN, "typed_keys_total_order.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split(":", 1)
        d[k.strip()] = v.split()
    return d


def pin_typed_golden(o):
    """Hand-worked orders of float (IEEE totalOrder) and signed keys."""
    g = load_typed_golden()
    for name, dt, raw in (("f32_keys", np.float32, np.uint32), ("f64_keys", np.float64, np.uint64)):
        bits = np.array([int(x, 16) for x in g[name]], dtype=raw)
        keys = bits.view(dt)
        vals = np.arange(keys.size, dtype=np.uint32)
        ok, ov = o.stable_sort_typed(keys, vals)
        assert list(ov) == [int(x) for x in g["float_sorted_vals"]], name
        assert np.array_equal(ok.view(raw), bits[ov]), name  # encodings come back unchanged
    for name, dt in (("i32_keys", np.int32), ("i64_keys", np.int64)):
        keys = np.array([int(x) for x in g[name]], dtype=dt)
        vals = np.arange(keys.size, dtype=np.uint64)
        ok, ov = o.stable_sort_typed(keys, vals)
        assert list(ov) == [int(x) for x in g["int_sorted_vals"]], name
        assert np.array_equal(ok, keys[ov.astype(np.int64)]), name


def pin_typed_numpy(o):
    """Signed keys, and finite nonzero floats (where totalOrder is the numeric order),
    against numpy's stable argsort."""
    rng = np.random.default_rng(11)
    for dt in (np.int32, np.int64):
        info = np.iinfo(dt)
        k = rng.integers(info.min, info.max, size=5000, dtype=dt, endpoint=True)
        k[:4] = [info.min, info.max, -1, 0]
        k[4:400] = k[4:400] % 7  # repeats
        ok, ov = o.stable_sort_typed(k, np.arange(k.size, dtype=np.uint32))
        ref = np.argsort(k, kind="stable")
        assert np.array_equal(ov, ref.astype(np.uint32)) and np.array_equal(ok, k[ref]), dt
    for dt in (np.float32, np.float64):
        k = (rng.standard_normal(5000) * rng.choice([1e-30, 1.0, 1e30], 5000)).astype(dt)
        k[k == 0] = 1
        k[:300] = np.round(k[:300])  # repeats
        k[k == 0] = 2
        ok, ov = o.stable_sort_typed(k, np.arange(k.size, dtype=np.uint32))
        ref = np.argsort(k, kind="stable")
        assert np.array_equal(ov, ref.astype(np.uint32)), dt
    # Unsigned keys through the typed entry give the plain definition.
    k = rng.integers(0, 1 << 32, size=3000, dtype=np.uint32)
    assert np.array_equal(o.stable_sort_typed(k)[0], o.stable_sort(k)[0])


def pin_overflow_enumeration(o):
    """Eq. 2 against the expected overflow computed over every one of the M^N equally
    likely ways to deal N records into M buckets of N/M slots (tiny N)."""
    import itertools
    from fractions import Fraction
    for N, M in ((1, 2), (2, 2), (3, 2), (5, 2), (7, 2), (4, 3), (6, 3), (8, 2), (5, 4), (7, 4)):
        cap = Fraction(N, M)
        total = Fraction(0)
        for deal in itertools.product(range(M), repeat=N):
            counts = [deal.count(b) for b in range(M)]
            total += sum(max(Fraction(0), c - cap) for c in counts)
        exact = total / (M ** N) / N
        assert abs(o.overflow_fraction(N, M) - float(exact)) < 1e-12, (N, M)


def pin_overflow_monte_carlo(o):
    """Eq. 2 against simulation (multinomial deals), and its large-N limit."""
    import math
    rng = np.random.default_rng(5)
    for N, M, trials in ((1000, 256, 4000), (65536, 256, 400), (300, 16, 4000)):
        counts = rng.multinomial(N, [1.0 / M] * M, size=trials)
        frac = np.maximum(counts - N / M, 0).sum(axis=1) / N
        mean, sem = frac.mean(), frac.std() / math.sqrt(trials)
        assert abs(o.overflow_fraction(N, M) - mean) < 5 * sem + 1e-12, (N, M)
    N = 1 << 24
    assert abs(o.overflow_fraction(N, 256) / math.sqrt(255 / (2 * math.pi * N)) - 1) < 1e-3


def pin_parallel(o):
    """The multi-threaded variant against numpy's stable argsort (an independent
    library) on heavy duplicates, for thread counts below, at and above the record
    count, and on the brute-force alphabet."""
    rng = np.random.default_rng(17)
    for n in (0, 1, 2, 5, 64, 1000, 65_537):
        for threads in (1, 2, 3, 8, 16, 70):
            k = rng.integers(0, 40, n, dtype=np.uint32)
            v = workloads.index_payload(n)
            ref = np.argsort(k, kind="stable")
            pk, pv = o.stable_sort_parallel(k, v, threads)
            assert np.array_equal(pv, ref) and np.array_equal(pk, k[ref]), (n, threads)
    for keys in itertools.product(range(3), repeat=6):
        k = np.array(keys, dtype=np.uint64)
        v = workloads.index_payload(k.size, 64)
        (perm,) = brute_stable_permutation(keys)
        pk, pv = o.stable_sort_parallel(k, v, 3)
        assert list(pv) == list(perm), keys


ALL_PINS = [pin_bruteforce_small_alphabet, pin_bruteforce_extremes, pin_numpy,
            pin_special_cases, pin_golden, pin_properties, pin_rank_formula,
            pin_typed_golden, pin_typed_numpy, pin_overflow_enumeration,
            pin_overflow_monte_carlo, pin_parallel]


# --------------------------------------------------------------------------------------
# The pins on the real oracle.
# --------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def o():
    return oracle.get()


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin(o, pin):
    pin(o)


def test_count_matches_bincount(o):
    for bits_k in (32, 64):
        k = workloads.make_keys("uniform", 100_000, bits_k, 1)
        for shift, bits in ((0, 8), (8, 8), (bits_k - 8, 8), (3, 5), (bits_k - 11, 11)):
            d = ((k >> k.dtype.type(shift)) & k.dtype.type((1 << bits) - 1)).astype(np.int64)
            assert np.array_equal(o.count(k, shift, bits), np.bincount(d, minlength=1 << bits))


def test_deal_is_stable_partition(o):
    for bits_k in (32, 64):
        k = workloads.make_keys("zipf", 60_000, bits_k, 2)
        v = workloads.index_payload(k.size, bits_k)
        for shift in range(0, bits_k, 8):
            d = (k >> k.dtype.type(shift)) & k.dtype.type(255)
            ref = np.argsort(d, kind="stable")
            dk, dv = o.deal(k, v, shift, 8)
            assert np.array_equal(dv, v[ref]) and np.array_equal(dk, k[ref])


@pytest.mark.parametrize("bits", [1, 4, 8, 11])
def test_lsd_equals_definition(o, bits):
    for dist, kb in (("uniform", 32), ("normal", 32), ("uniform", 64), ("skewed", 64)):
        k = workloads.make_keys(dist, 20_000, kb, bits)
        v = workloads.index_payload(k.size, kb)
        ref = np.argsort(k, kind="stable")
        lk, lv = o.lsd_sort(k, v, bits)
        assert np.array_equal(lv, ref) and np.array_equal(lk, k[ref])


@pytest.mark.parametrize("divert", [1, 16, 300, 5000])
def test_dfr_steps_equal_definition(o, divert):
    for dist, kb in (("uniform", 32), ("zipf", 32), ("few", 32), ("normal", 32),
                     ("skewed", 64), ("equal", 64), ("narrow", 64)):
        k = workloads.make_keys(dist, 30_000, kb, divert)
        v = workloads.index_payload(k.size, kb)
        ref = np.argsort(k, kind="stable")
        dk, dv = o.dfr_sort(k, v, 8, divert)
        assert np.array_equal(dv, ref) and np.array_equal(dk, k[ref]), dist


def test_bucket_starts(o):
    k = np.sort(workloads.make_keys("uniform", 50_000, 32, 4))
    for lo_bit in (0, 8, 16, 24, 31):
        pre = k >> np.uint32(lo_bit)
        ref = np.flatnonzero(np.r_[True, pre[1:] != pre[:-1]])
        assert np.array_equal(o.bucket_starts(k, lo_bit), ref)


def test_segmented(o):
    lens = workloads.batch_lengths(300, 1, 2000, 3)
    lens[5] = 0
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    k = workloads.make_keys("zipf", n, 32, 9)
    v = workloads.index_payload(n)
    sk, sv = o.segmented_sort(k, v, off)
    for s in range(lens.size):
        a, b = int(off[s]), int(off[s + 1])
        ref = np.argsort(k[a:b], kind="stable") + a
        assert np.array_equal(sv[a:b], ref) and np.array_equal(sk[a:b], k[ref])


def test_checker_catches_each_broken_property(o):
    k = workloads.make_keys("few", 1000, 32, 1)
    ok, ov = o.stable_sort(k, workloads.index_payload(1000))
    assert o.check_index_payload(k, ok, ov) is None
    ties = np.flatnonzero(ok[1:] == ok[:-1])[0]
    bad = ov.copy(); bad[4] = bad[3]
    assert o.check_index_payload(k, ok, bad)[1] == 1
    badk = ok.copy(); badk[10] ^= np.uint32(1)
    assert o.check_index_payload(k, badk, ov)[1] in (2, 3)
    swapped_k, swapped_v = ok.copy(), ov.copy()
    i = np.flatnonzero(ok[1:] != ok[:-1])[0]
    swapped_k[[i, i + 1]] = swapped_k[[i + 1, i]]
    swapped_v[[i, i + 1]] = swapped_v[[i + 1, i]]
    assert o.check_index_payload(k, swapped_k, swapped_v)[1] == 3
    unstable_v = ov.copy()
    unstable_v[[ties, ties + 1]] = unstable_v[[ties + 1, ties]]
    assert o.check_index_payload(k, ok, unstable_v)[1] == 4


# --------------------------------------------------------------------------------------
# Planted mistakes: each mutant build must fail at least one pin.
# --------------------------------------------------------------------------------------

MUTANTS = ["ORACLE_PLANT_REVERSED_TIES", "ORACLE_PLANT_SIGNED_COMPARE",
           "ORACLE_PLANT_DROP_LAST", "ORACLE_PLANT_INCLUSIVE_SCAN",
           "ORACLE_PLANT_FLOAT_NO_REVERSE", "ORACLE_PLANT_OVERFLOW_EXTRA_TERM",
           "ORACLE_PLANT_MERGE_RIGHT_FIRST"]


@pytest.mark.parametrize("mutant", MUTANTS)
def test_planted_mistakes(tmp_path, mutant):
    path = oracle.build(str(tmp_path / f"lib_{mutant}.so"), defines=(mutant,))
    bad = oracle.Oracle(path)
    failed = []
    for pin in ALL_PINS:
        try:
            pin(bad)
        except (AssertionError, RuntimeError):
            failed.append(pin.__name__)
    assert failed, f"no pin caught {mutant}"
