"""Launch settings (digit width, deal tile, diversion threshold, window width) and the
autotuner: none of them may change the result, which stays the stable sort computed
by the oracle, bit for bit."""
from __future__ import annotations

import json
import os

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


def sort_with(torch, ctx, k, v, off, opts):
    for name, val in opts.items():
        ctx.set_option(name, val)
    try:
        dk = torch.from_numpy(k).cuda()
        dv = torch.from_numpy(v).cuda()
        if off is None:
            ctx.sort_(dk, dv)
        else:
            ctx.sort_segmented_(dk, dv, off)
        torch.cuda.synchronize()
        return dk.cpu().numpy(), dv.cpu().numpy(), ctx.stats()
    finally:
        for name in opts:
            ctx.set_option(name, 0)


def reference(o, k, v, off):
    return o.stable_sort(k, v) if off is None else o.segmented_sort(k, v, off)


SHAPES = ["plain", "recursion", "segmented"]


def make(shape, bits, seed):
    if shape == "plain":
        n, off = (1 << 21) + 7, None
    elif shape == "recursion":
        n, off = (1 << 22) + 3, None
    else:
        lens = workloads.batch_lengths(500, 16, 1 << 17, seed)
        off = workloads.segment_offsets(lens)
        n = int(off[-1])
    dist = "normal" if shape == "recursion" else "uniform"
    return workloads.make_keys(dist, n, bits, seed), workloads.index_payload(n, bits), off


@pytest.mark.parametrize("rb", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("shape", SHAPES)
def test_radix_bits(env, o, rb, shape):
    torch, dfr, ctx = env
    k, v, off = make(shape, 32, rb)
    say("radix_bits", rb, shape, k.size)
    opts = {"radix_bits": rb}
    if shape == "recursion":
        opts["force_top_digits"] = 1
    sk, sv, st = sort_with(torch, ctx, k, v, off, opts)
    rk, rv = reference(o, k, v, off)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("half", [False, True])
@pytest.mark.parametrize("shape", SHAPES)
def test_tile_records(env, o, bits, half, shape):
    torch, dfr, ctx = env
    kb = bits // 8
    tile = dfr.deal_tile_records(kb, kb) // (2 if half else 1)
    k, v, off = make(shape, bits, 3)
    say("tile_records", bits, tile, shape, k.size)
    sk, sv, st = sort_with(torch, ctx, k, v, off, {"tile_records": tile})
    rk, rv = reference(o, k, v, off)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st


@pytest.mark.parametrize("window", [16, 100, 1024, 1 << 20])
@pytest.mark.parametrize("divert", [1, 700, 1 << 20])
def test_window_and_divert(env, o, window, divert):
    torch, dfr, ctx = env
    k, v, off = make("segmented", 32, 5)
    say("window/divert", window, divert, k.size)
    sk, sv, st = sort_with(torch, ctx, k, v, off, {"window_records": window, "divert_records": divert})
    rk, rv = reference(o, k, v, off)
    assert np.array_equal(sk, rk) and np.array_equal(sv, rv), st


def test_bad_option_values(env):
    torch, dfr, ctx = env
    for name, val in (("radix_bits", 3), ("radix_bits", 9), ("tile_records", -1),
                      ("window_records", -5)):
        with pytest.raises(dfr.DfrError) as e:
            ctx.set_option(name, val)
        assert e.value.status == dfr.E_INVALID_ARG


def test_autotune_segmented(env, o, tmp_path):
    torch, dfr, ctx = env
    lens = workloads.batch_lengths(2000, 16, 1 << 16, 8)
    off = workloads.segment_offsets(lens)
    n = int(off[-1])
    k = workloads.make_keys("zipf", n, 32, 8)
    v = workloads.index_payload(n)
    dk, dv = torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda()
    say("autotune", n)
    t = ctx.autotune(dk, dv, off, reps=1)
    torch.cuda.synchronize()
    # The tuner only reads its inputs.
    assert np.array_equal(dk.cpu().numpy(), k) and np.array_equal(dv.cpu().numpy(), v)
    assert t["ms"] > 0 and t["ms_default"] > 0 and t["ms"] <= t["ms_default"] * 1.0001
    cls = dfr.size_class(off)
    assert ctx.get_tune(4, 4, cls)["radix_bits"] == t["radix_bits"]
    # The stored setting is used by the next call of that class; the result is the oracle's.
    ctx.sort_segmented_(dk, dv, off)
    torch.cuda.synchronize()
    rk, rv = o.segmented_sort(k, v, off)
    assert np.array_equal(dk.cpu().numpy(), rk) and np.array_equal(dv.cpu().numpy(), rv)
    # Save, clear, load.
    path = os.path.join(tmp_path, "tune.json")
    ctx.save_tuning(path)
    saved = json.load(open(path))
    assert any(e["size_class"] == cls for e in saved["entries"])
    ctx.set_tune(4, 4, cls, None)
    assert ctx.get_tune(4, 4, cls) is None
    assert ctx.load_tuning(path) == len(saved["entries"])
    assert ctx.get_tune(4, 4, cls)["tile_records"] == t["tile_records"]
    with pytest.raises(dfr.DfrError):
        ctx.set_tune(4, 4, cls, dict(t, tile_records=12345))
    ctx.set_tune(4, 4, cls, None)
