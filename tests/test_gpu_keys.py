"""Signed and floating-point keys on the GPU against the oracle's typed stable sort
(two's-complement order; IEEE 754 totalOrder), compared bit for bit on the encodings."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2207_14334_amd as dfr
    assert torch.cuda.is_available()
    ctx = dfr.Context(0)
    yield torch, dfr, ctx
    ctx.close()


@pytest.fixture(scope="module")
def o():
    return oracle.get()


RAW = {np.int32: np.uint32, np.int64: np.uint64, np.float32: np.uint32, np.float64: np.uint64}


def make(dt, n, seed):
    """Keys of dtype dt: the whole encoding range, repeats, and the special values."""
    raw = RAW[dt]
    bits = workloads.make_keys("uniform", n, 8 * np.dtype(raw).itemsize, seed)
    k = bits.view(dt).copy()
    rng = np.random.default_rng(seed)
    if np.issubdtype(dt, np.floating):
        finfo = np.finfo(dt)
        special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, finfo.tiny,
                            -finfo.tiny, finfo.max, -finfo.max, 1.0, -1.0,
                            finfo.smallest_subnormal, -finfo.smallest_subnormal], dtype=dt)
        m = max(1, n // 5)
        k[rng.integers(0, n, m)] = special[rng.integers(0, special.size, m)]
        # Finite values in a narrow range, with many repeats.
        m2 = max(1, n // 4)
        k[rng.integers(0, n, m2)] = np.round(rng.standard_normal(m2) * 100).astype(dt)
    else:
        info = np.iinfo(dt)
        special = np.array([info.min, info.max, -1, 0, 1], dtype=dt)
        m = max(1, n // 5)
        k[rng.integers(0, n, m)] = special[rng.integers(0, special.size, m)]
        m2 = max(1, n // 4)
        k[rng.integers(0, n, m2)] = rng.integers(-50, 50, m2).astype(dt)
    return k


SIZES = [1, 2, 1000, 3 * 8192 + 77, (1 << 20) + 5]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dt", [np.int32, np.int64, np.float32, np.float64], ids=lambda d: d.__name__)
@pytest.mark.parametrize("vdt", [None, np.uint32, np.uint64], ids=["keyonly", "v32", "v64"])
def test_typed_plain(env, o, n, dt, vdt):
    torch, dfr, ctx = env
    k = make(dt, n, n + 3)
    v = None if vdt is None else np.arange(n, dtype=vdt)
    say("typed", dt.__name__, vdt, n)
    dk = torch.from_numpy(k).cuda()
    dv = None if v is None else torch.from_numpy(v).cuda()
    ctx.sort_(dk, dv)
    torch.cuda.synchronize()
    rk, rv = o.stable_sort_typed(k, v)
    raw = RAW[dt]
    assert np.array_equal(dk.cpu().numpy().view(raw), rk.view(raw))
    if v is not None:
        assert np.array_equal(dv.cpu().numpy(), rv)


@pytest.mark.parametrize("dt", [np.int32, np.float32, np.int64, np.float64], ids=lambda d: d.__name__)
def test_typed_large(env, o, dt):
    """Several levels and both word forms of the local sort."""
    torch, dfr, ctx = env
    n = (1 << 23) + 11
    k = make(dt, n, 99)
    v = np.arange(n, dtype=np.uint32)
    say("typed large", dt.__name__, n)
    dk, dv = torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda()
    ctx.sort_(dk, dv)
    torch.cuda.synchronize()
    rk, rv = o.stable_sort_typed(k, v)
    raw = RAW[dt]
    assert np.array_equal(dk.cpu().numpy().view(raw), rk.view(raw))
    assert np.array_equal(dv.cpu().numpy(), rv)


@pytest.mark.parametrize("dt", [np.int32, np.int64, np.float32, np.float64], ids=lambda d: d.__name__)
def test_typed_segmented(env, o, dt):
    torch, dfr, ctx = env
    lens = workloads.batch_lengths(300, 1, 60000, 5)
    lens[7] = 0
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    k = make(dt, n, 17)
    v = np.arange(n, dtype=np.uint64)
    say("typed segmented", dt.__name__, n)
    dk, dv = torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda()
    ctx.sort_segmented_(dk, dv, off)
    torch.cuda.synchronize()
    raw = RAW[dt]
    ok, ov = dk.cpu().numpy(), dv.cpu().numpy()
    for s in range(lens.size):
        a, b = int(off[s]), int(off[s + 1])
        rk, rv = o.stable_sort_typed(k[a:b], v[a:b])
        assert np.array_equal(ok[a:b].view(raw), rk.view(raw)), s
        assert np.array_equal(ov[a:b], rv), s


def test_typed_argument_errors(env):
    torch, dfr, ctx = env
    import ctypes
    k = torch.from_numpy(np.arange(10, dtype=np.float32)).cuda()
    L = dfr.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.dfr_sort_keys(ctx._h, 6, k.data_ptr(), None, 0, 10, None, 0, s) == dfr.E_INVALID_ARG
    assert L.dfr_sort_keys(ctx._h, dfr.KEY_F32, k.data_ptr(), None, 4, 10, None, 0, s) == dfr.E_INVALID_ARG
    assert L.dfr_sort_keys(ctx._h, dfr.KEY_F32, k.data_ptr(), None, 3, 10, None, 0, s) == dfr.E_INVALID_ARG
    # Untouched after an argument error.
    assert np.array_equal(k.cpu().numpy(), np.arange(10, dtype=np.float32))
