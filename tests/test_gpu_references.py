"""The bandwidth references the benchmark times the passes against: the library's
streaming copy (every byte read and written once, like a deal or a local sort) and its
streaming read (every byte read once, like a count).  Each must do exactly its job: the
copy reproduces its source, and the read's XOR of all 32-bit words equals numpy's."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2207_14334_amd as dfr
    assert torch.cuda.is_available()
    ctx = dfr.Context(0)
    yield torch, dfr, ctx
    ctx.close()


SIZES = [0, 16, 4096, 16 * 12345, (1 << 24) + 48, (1 << 27) + 16]


@pytest.mark.parametrize("nbytes", SIZES)
def test_stream_read_checksum(env, nbytes):
    torch, dfr, ctx = env
    n = nbytes // 4
    print("[case] stream read", nbytes, flush=True)
    h = np.random.default_rng(nbytes).integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    src = torch.from_numpy(h.view(np.int32)).cuda()
    out = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    ctx.stream_read(src, out)
    torch.cuda.synchronize()
    want = int(np.bitwise_xor.reduce(h)) if n else 0
    assert int(out.cpu().numpy().view(np.uint32)[0]) == want


@pytest.mark.parametrize("nbytes", SIZES[1:])
def test_stream_copy_reproduces(env, nbytes):
    torch, dfr, ctx = env
    n = nbytes // 4
    print("[case] stream copy", nbytes, flush=True)
    src = torch.randint(-(1 << 31), (1 << 31) - 1, (n,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    ctx.stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_stream_read_rejects_bad_sizes(env):
    torch, dfr, ctx = env
    src = torch.zeros(5, dtype=torch.int32, device="cuda")  # 20 bytes: not a multiple of 16
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError):
        ctx.stream_read(src, out)
    with pytest.raises(ValueError):
        ctx.stream_read(torch.zeros(4, dtype=torch.int32, device="cuda"),
                        torch.zeros(2, dtype=torch.int32, device="cuda"))
