"""The seeded input generators: determinism and the shapes the paper's workloads have."""
from __future__ import annotations

import numpy as np

import workloads


def test_deterministic_per_seed():
    for dist in workloads.DISTS:
        bits = 64 if dist == "skewed" else 32
        a = workloads.make_keys(dist, 100_000, bits, 3)
        b = workloads.make_keys(dist, 100_000, bits, 3)
        c = workloads.make_keys(dist, 100_000, bits, 4)
        assert np.array_equal(a, b), dist
        if dist != "equal":
            assert not np.array_equal(a, c), dist


def test_zipf_mass():
    k = workloads.make_keys("zipf", 1 << 22, 32, 0)
    p0 = np.mean(k == 0)
    p16 = np.mean(k < (1 << 16))
    assert abs(p0 - 0.105) < 0.01, p0      # P(key = 0) ~ 10.5% for s = 1.1
    assert abs(p16 - 0.77) < 0.02, p16     # P(key < 2^16) ~ 77%


def test_normal_moments():
    k = workloads.make_keys("normal", 1 << 22, 32, 0).astype(np.float64)
    assert abs(k.mean() / 2**31 - 1) < 1e-3
    assert abs(k.std() / 2**28 - 1) < 1e-2


def test_few_and_skewed_shapes():
    few = workloads.make_keys("few", 1 << 20, 32, 0)
    assert np.unique(few).size <= 256
    sk = workloads.make_keys("skewed", 1 << 20, 64, 0)
    assert np.unique(sk >> np.uint64(48)).size <= 4


def test_batch_lengths_log_uniform():
    lens = workloads.batch_lengths(20000, 16, 1 << 20, 0)
    assert lens.min() >= 16 and lens.max() <= 1 << 20
    # log-uniform: half of the arrays below 4096 = 16 * 2^8
    frac = np.mean(lens < 4096)
    assert abs(frac - 0.5) < 0.02, frac  # ln(4096/16) / ln(2^20/16) = 8/16


def test_request_stream_mix():
    s = workloads.request_stream(2000, 1.0, 1 << 10, 1 << 24, 0.3, 0.5, 0)
    wide = np.mean([r[2] == 64 for r in s])
    zipf = np.mean([r[3] == "zipf" for r in s])
    assert abs(wide - 0.3) < 0.04 and abs(zipf - 0.5) < 0.04
    arrive = np.array([r[0] for r in s])
    assert np.all(np.diff(arrive) >= 0) and arrive[0] == 0.0


def test_permutation_keys_are_distinct_and_invertible():
    """k_i = (a i + b) mod 2^32 with a odd: distinct keys, and the index of a key is
    recovered as (k - b) a^-1 mod 2^32 (what the size-limit test relies on)."""
    n = 1 << 18
    k, a, b = workloads.permutation_keys(n, 9)
    assert a % 2 == 1 and np.unique(k).size == n
    a_inv = pow(a, -1, 1 << 32)
    idx = ((k.astype(np.uint64) - np.uint64(b)) * np.uint64(a_inv)) & np.uint64(0xFFFFFFFF)
    assert np.array_equal(idx, np.arange(n, dtype=np.uint64))
    k2, a2, b2 = workloads.permutation_keys(n, 9)
    assert np.array_equal(k, k2) and (a, b) == (a2, b2)


def test_device_generators_shapes():
    """The torch-drawn benchmark inputs have the shapes of make_keys' (run here on the
    CPU device): Zipf(1.1) mass at 0 and below 2^16, normal moments, the uniform range,
    determinism per seed, and the index payload."""
    import torch
    n = 1 << 21
    z = workloads.make_keys_device("zipf", n, 32, 0, device="cpu")
    zi = z.view(torch.int32).numpy().view(np.uint32)
    assert abs(np.mean(zi == 0) - 0.105) < 0.01 and abs(np.mean(zi < (1 << 16)) - 0.77) < 0.02
    g = workloads.make_keys_device("normal", n, 32, 0, device="cpu").view(torch.int32).numpy()
    g = g.view(np.uint32).astype(np.float64)
    assert abs(g.mean() / 2**31 - 1) < 1e-3 and abs(g.std() / 2**28 - 1) < 1e-2
    u = workloads.make_keys_device("uniform", n, 32, 0, device="cpu").view(torch.int32).numpy()
    u = u.view(np.uint32).astype(np.float64)
    assert abs(u.mean() / 2**31 - 1) < 5e-3 and u.max() > 2**32 * 0.999
    u2 = workloads.make_keys_device("uniform", n, 32, 0, device="cpu")
    assert torch.equal(u2, workloads.make_keys_device("uniform", n, 32, 0, device="cpu"))
    w = workloads.make_keys_device("uniform", 1000, 64, 1, device="cpu").view(torch.int64).numpy()
    assert w.view(np.uint64).max() > (1 << 63)
    v = workloads.index_payload_device(10, 32, 5, device="cpu").view(torch.int32).numpy()
    assert list(v) == list(range(5, 15))
