"""The allocation-free entry point (dfr_sort_noalloc), called through the C ABI, against
the existing plain sort (dfr_sort_u32/u64) on the same inputs, bit for bit, on two calls
in a row with the second smaller; plus its size limit and that it allocates nothing.
Collected last: it shares the device's fixed scratch array with nothing else here."""
from __future__ import annotations

import ctypes

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
    torch.cuda.set_device(0)
    return torch, dfr


def noalloc(dfr, ctx, dk, dv, n, kb, vb, stream):
    return dfr.lib().dfr_sort_noalloc(ctx._h, dk.data_ptr(), dv.data_ptr() if dv is not None else None,
                                      n, kb, vb, ctypes.c_void_p(stream.cuda_stream))


def plain(dfr, ctx, dk, dv, n, kb, stream):
    f = dfr.lib().dfr_sort_u32 if kb == 4 else dfr.lib().dfr_sort_u64
    return f(ctx._h, dk.data_ptr(), dv.data_ptr() if dv is not None else None, n, None, 0,
             ctypes.c_void_p(stream.cuda_stream))


CASES = [
    # (key bits, payload bits, distribution, first n, second n)
    (32, 32, "uniform", 1 << 22, 100_003),
    (32, 32, "zipf", 1 << 22, (1 << 20) + 7),
    (32, 0, "few", (1 << 21) + 3, 4097),
    (64, 64, "skewed", 1 << 22, 70_001),
    (64, 64, "normal", (1 << 22) - 1, 8193),
    (32, 64, "uniform", 3_000_001, 2),
]


@pytest.mark.parametrize("bits,vbits,dist,n1,n2", CASES,
                         ids=[f"u{b}v{v}-{d}-{a}-{c}" for b, v, d, a, c in CASES])
def test_noalloc_matches_plain(env, bits, vbits, dist, n1, n2):
    torch, dfr = env
    kb, vb = bits // 8, vbits // 8
    stream = torch.cuda.current_stream()
    a = dfr.Context(0)  # the allocation-free calls
    b = dfr.Context(0)  # the plain calls
    try:
        for call, n in enumerate((n1, n2)):
            k = workloads.make_keys(dist, n, bits, 40 + call)
            v = workloads.index_payload(n, vbits) if vb else None
            say("noalloc", bits, vbits, dist, n, "call", call)
            dk = torch.from_numpy(k).cuda()
            dv = torch.from_numpy(v).cuda() if v is not None else None
            pk = dk.clone()
            pv = dv.clone() if dv is not None else None
            # The existing entry point first (it also brings the kernels' own runtime
            # resources into being), then the allocation-free one.
            if vb == kb or vb == 0:
                assert plain(dfr, b, pk, pv, n, kb, stream) == dfr.OK, b.last_error()
            else:  # a payload of another width: the typed entry point on unsigned keys
                kt = dfr.KEY_U32 if kb == 4 else dfr.KEY_U64
                assert dfr.lib().dfr_sort_keys(b._h, kt, pk.data_ptr(), pv.data_ptr(), vb, n, None, 0,
                                               ctypes.c_void_p(stream.cuda_stream)) == dfr.OK
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            assert noalloc(dfr, a, dk, dv, n, kb, vb, stream) == dfr.OK, a.last_error()
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            # Nothing allocated on the device (a first ordinary sort on a fresh context
            # takes a temp buffer and a scratch arena of 16 MiB or more).
            assert free0 - free1 < (4 << 20), (free0, free1)
            assert torch.equal(dk, pk), (n, call)
            if dv is not None:
                assert torch.equal(dv, pv), (n, call)
                assert oracle.get().check_index_payload(k, dk.cpu().numpy(), dv.cpu().numpy()) is None
    finally:
        a.close()
        b.close()


def test_noalloc_limits(env):
    torch, dfr = env
    stream = torch.cuda.current_stream()
    with dfr.Context(0) as ctx:
        k = torch.from_numpy(np.arange(16, dtype=np.uint32)).cuda()
        assert noalloc(dfr, ctx, k, None, dfr.NOALLOC_MAX_RECORDS + 1, 4, 0, stream) == dfr.E_TOO_LARGE
        assert noalloc(dfr, ctx, k, None, 16, 3, 0, stream) == dfr.E_INVALID_ARG
        assert noalloc(dfr, ctx, k, None, 1, 4, 0, stream) == dfr.OK
        torch.cuda.synchronize()
        assert np.array_equal(k.cpu().numpy(), np.arange(16, dtype=np.uint32))
