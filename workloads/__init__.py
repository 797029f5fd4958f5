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


# --------------------------------------------------------------------------------------
# The same shapes drawn on the GPU (torch's Philox generator, seeded), for benchmark
# inputs of billions of keys that numpy would take minutes to draw.  Tests use the numpy
# generators above.
# --------------------------------------------------------------------------------------

def _torch_gen(seed: int, stream: int, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed((seed * 1_000_003 + stream) & ((1 << 63) - 1))
    return g


def _as_unsigned(x, key_bits):
    """int64 tensor of values in [0, 2^key_bits) -> uint32/uint64 tensor of those values."""
    import torch
    if key_bits == 64:
        return x.view(torch.uint64)
    x = torch.where(x >= (1 << 31), x - (1 << 32), x).to(torch.int32)
    return x.view(torch.uint32)


def make_keys_device(dist: str, n: int, key_bits: int = 32, seed: int = 0, device="cuda"):
    """``n`` keys of distribution ``dist`` ("uniform", "normal" or "zipf", with the
    parameters of make_keys) drawn on the GPU; a uint32/uint64 tensor."""
    import torch
    if key_bits not in (32, 64):
        raise ValueError("key_bits must be 32 or 64")
    out = torch.empty(n, dtype=torch.uint32 if key_bits == 32 else torch.uint64, device=device)
    g = _torch_gen(seed, 7, device)
    step = 1 << 26
    if dist == "zipf":
        # Zipf(s) by Devroye's rejection method (Non-Uniform Random Variate Generation,
        # 1986, ch. X.6): X = floor(U^(-1/(s-1))), accepted when
        # V X (T - 1) / (b - 1) <= T / b with T = (1 + 1/X)^(s-1), b = 2^(s-1);
        # ranks above the key range are redrawn, as make_keys does; key = rank - 1.
        s_, limit = 1.1, float(1 << 32) if key_bits == 32 else float(1 << 63)
        am1 = s_ - 1.0
        b = 2.0 ** am1
        filled = 0
        while filled < n:
            m = min(step, int((n - filled) * 1.4) + 4096)
            u = 1.0 - torch.rand(m, dtype=torch.float64, generator=g, device=device)
            v = torch.rand(m, dtype=torch.float64, generator=g, device=device)
            x = torch.floor(u.pow(-1.0 / am1))
            t = (1.0 + 1.0 / x).pow(am1)
            ok = (x >= 1.0) & (x <= limit) & (v * x * (t - 1.0) / (b - 1.0) <= t / b)
            r = x[ok][: n - filled]
            k = r.to(torch.int64) - 1 if key_bits == 32 else (r - 1.0).to(torch.int64)
            out[filled:filled + k.numel()] = _as_unsigned(k, key_bits)
            filled += k.numel()
        return out
    for lo in range(0, n, step):
        m = min(step, n - lo)
        if dist == "uniform":
            if key_bits == 32:
                x = torch.randint(0, 1 << 32, (m,), dtype=torch.int64, generator=g, device=device)
            else:
                x = torch.randint(-(1 << 63), (1 << 63) - 1, (m,), dtype=torch.int64, generator=g,
                                  device=device)
                out[lo:lo + m] = x.view(torch.uint64)
                continue
        elif dist == "normal":
            mean, sd = float(2 ** (key_bits - 1)), float(2 ** (key_bits - 4))
            y = torch.normal(mean, sd, (m,), dtype=torch.float64, generator=g, device=device)
            if key_bits == 64:
                # Rounded and clipped to the key range, taken as (value - 2^63) in int64,
                # then the sign bit flipped: the value's 64-bit pattern.
                z = torch.clamp(torch.round(y) - 2.0 ** 63, -(2.0 ** 63), 2.0 ** 63 - 1024.0)
                out[lo:lo + m] = (z.to(torch.int64) ^ (-(1 << 63))).view(torch.uint64)
                continue
            x = torch.clamp(torch.round(y), 0.0, float(2 ** 32 - 1)).to(torch.int64)
        else:
            raise ValueError(f"distribution {dist!r} is not drawn on the GPU")
        out[lo:lo + m] = _as_unsigned(x, key_bits)
    return out


def index_payload_device(n: int, val_bits: int = 32, offset: int = 0, device="cuda"):
    """The index payload v_i = offset + i as a uint32/uint64 GPU tensor."""
    import torch
    x = torch.arange(offset, offset + n, dtype=torch.int64, device=device)
    return _as_unsigned(x, val_bits) if val_bits == 32 else x.view(torch.uint64)


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
