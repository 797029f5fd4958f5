"""Seeded synthetic inputs shaped like the paper's workloads.

The paper times uniform, normal and Zipf integer keys (Sec. 5, experiments paragraph;
figure captions of Sec. 3.1 and Sec. 5).  No dataset is involved, so every input here is
drawn from numpy's PCG64 generator with an explicit seed.  This module holds only input
generation: none of the sort's arithmetic.  Both the GPU tests and the CPU oracle take
their inputs from here.

Key distributions (``make_keys``):

* ``uniform``   -- i.i.d. uniform over the whole key range.
* ``normal``    -- normal with mean 2^(w-1) and sd 2^(w-4), rounded and clipped to the
                   key range (w = key bits).  For 32-bit keys: mean 2^31, sd 2^28.
* ``zipf``      -- Zipf(s=1.1) ranks r >= 1, redrawn while r > 2^32, key = r - 1 (drawn
                   in chunks of 2^22 from per-chunk child streams of the seed).
* ``sorted`` / ``reverse`` -- the uniform draw sorted ascending / descending.
* ``few``       -- 256 distinct values drawn uniformly, each key one of them.
* ``skewed``    -- 64-bit keys whose top 16 bits take only 4 values (drawn uniformly)
                   and whose low 48 bits are uniform.
* ``equal``     -- every key the same uniform draw.
* ``narrow``    -- keys spread over only the low ``narrow_bits`` bits (default 20).
"""
from __future__ import annotations

import os

import numpy as np

DISTS = ("uniform", "normal", "zipf", "sorted", "reverse", "few", "skewed", "equal", "narrow")

_CHUNK = 1 << 22


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def _uniform(rng, n, bits):
    if bits == 32:
        return rng.integers(0, 1 << 32, size=n, dtype=np.uint32)
    return rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)


def _zipf_chunk(seed, chunk, m, bits):
    """m Zipf(1.1) keys from the chunk's own stream (redrawn while the rank is too big)."""
    rng = _rng(seed, 1000 + chunk)
    limit = (1 << 32) if bits == 32 else (1 << 63)
    parts, got = [], 0
    while got < m:
        r = rng.zipf(1.1, size=m - got + (m - got) // 8 + 16)
        r = r[(r >= 1) & (r <= limit)][: m - got]
        parts.append(r)
        got += r.size
    return (np.concatenate(parts) - 1).astype(np.uint32 if bits == 32 else np.uint64)


def _zipf(seed, n, bits):
    # Chunks of 2^22 keys, each from its own child stream, drawn in parallel threads
    # (numpy releases the GIL while drawing); the result depends only on (seed, n).
    from concurrent.futures import ThreadPoolExecutor
    nch = (n + _CHUNK - 1) // _CHUNK
    sizes = [min(_CHUNK, n - c * _CHUNK) for c in range(nch)]
    workers = max(1, min(16, os.cpu_count() or 1, nch))
    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(lambda c: _zipf_chunk(seed, c, sizes[c], bits), range(nch)))
    return np.concatenate(parts) if parts else np.empty(0, np.uint32 if bits == 32 else np.uint64)


def make_keys(dist: str, n: int, key_bits: int = 32, seed: int = 0, *,
              narrow_bits: int = 20) -> np.ndarray:
    """Return ``n`` keys (uint32 when key_bits == 32, else uint64) of distribution ``dist``."""
    if key_bits not in (32, 64):
        raise ValueError("key_bits must be 32 or 64")
    dt = np.uint32 if key_bits == 32 else np.uint64
    rng = _rng(seed)
    if n == 0:
        return np.empty(0, dtype=dt)
    if dist == "uniform":
        return _uniform(rng, n, key_bits)
    if dist == "normal":
        mean, sd = float(2 ** (key_bits - 1)), float(2 ** (key_bits - 4))
        x = np.rint(rng.normal(mean, sd, size=n))
        hi = float(2 ** key_bits - 1)
        x = np.clip(x, 0.0, hi)
        if key_bits == 64:
            # float64 cannot hold every 64-bit integer; the top value saturates.
            out = np.empty(n, dtype=np.uint64)
            big = x >= 2.0 ** 63
            out[~big] = x[~big].astype(np.int64).astype(np.uint64)
            out[big] = (x[big] - 2.0 ** 63).astype(np.uint64) + np.uint64(1 << 63)
            return out
        return x.astype(np.uint32)
    if dist == "zipf":
        return _zipf(seed, n, key_bits)
    if dist == "sorted":
        return np.sort(_uniform(rng, n, key_bits))
    if dist == "reverse":
        return np.sort(_uniform(rng, n, key_bits))[::-1].copy()
    if dist == "few":
        pool = _uniform(rng, 256, key_bits)
        return pool[rng.integers(0, 256, size=n)]
    if dist == "skewed":
        if key_bits != 64:
            raise ValueError("skewed keys are 64-bit")
        top = rng.integers(0, 1 << 16, size=4, dtype=np.uint64)
        low = rng.integers(0, 1 << 48, size=n, dtype=np.uint64)
        return (top[rng.integers(0, 4, size=n)] << np.uint64(48)) | low
    if dist == "equal":
        return np.full(n, _uniform(rng, 1, key_bits)[0], dtype=dt)
    if dist == "narrow":
        return rng.integers(0, 1 << narrow_bits, size=n, dtype=dt)
    raise ValueError(f"unknown distribution {dist!r}")


def permutation_keys(n: int, seed: int = 0) -> tuple[np.ndarray, int, int]:
    """``n`` <= 2^32 distinct uint32 keys k_i = (a * i + b) mod 2^32 with a odd (a
    bijection of the 32-bit values, so the keys are distinct), a and b drawn from the
    seed; returns (keys, a, b).  Built in chunks, for inputs up to the 32-bit limit."""
    if n > 1 << 32:
        raise ValueError("at most 2^32 distinct 32-bit keys")
    rng = _rng(seed, 3)
    a = int(rng.integers(0, 1 << 31)) * 2 + 1
    b = int(rng.integers(0, 1 << 32))
    out = np.empty(n, dtype=np.uint32)
    step = 1 << 26
    for lo in range(0, n, step):
        i = np.arange(lo, min(n, lo + step), dtype=np.uint64)
        out[lo:lo + i.size] = ((i * np.uint64(a) + np.uint64(b)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return out, a, b


def index_payload(n: int, val_bits: int = 32) -> np.ndarray:
    """The payload v_i = i, which makes the stable sort checkable by its properties."""
    return np.arange(n, dtype=np.uint32 if val_bits == 32 else np.uint64)


def batch_lengths(count: int, lo: int, hi: int, seed: int = 0) -> np.ndarray:
    """``count`` array lengths, log-uniform in [lo, hi] (floor of exp(uniform))."""
    rng = _rng(seed, 1)
    x = np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))
    return np.clip(np.floor(x), lo, hi).astype(np.int64)


def segment_offsets(lengths) -> np.ndarray:
    """Offsets [0, l0, l0+l1, ...] of segments laid end to end."""
    lengths = np.asarray(lengths, dtype=np.uint64)
    off = np.zeros(lengths.size + 1, dtype=np.uint64)
    np.cumsum(lengths, out=off[1:])
    return off


def request_stream(count: int, rate_per_s: float, lo: int = 1 << 10, hi: int = 1 << 24,
                   frac_u64: float = 0.3, frac_zipf: float = 0.5, seed: int = 0):
    """A Poisson stream of sort requests: (arrival_s, n, key_bits, dist) tuples."""
    rng = _rng(seed, 2)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrive = np.cumsum(gaps) - gaps[0]
    sizes = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    wide = rng.uniform(size=count) < frac_u64
    zipf = rng.uniform(size=count) < frac_zipf
    return [(float(arrive[i]), int(sizes[i]), 64 if wide[i] else 32,
             "zipf" if zipf[i] else "uniform") for i in range(count)]
