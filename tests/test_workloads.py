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
