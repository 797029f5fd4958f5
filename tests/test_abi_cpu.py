"""Host-side checks of the C ABI: the library loads without a GPU, exports every entry
point that include/dfr.h declares, validates arguments before touching the device, and
its planner (pure host code) picks the number of top digits as documented."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2207_14334_amd as dfr
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfr.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(dfr.LIB_PATH):
        from paper_2207_14334_amd import build
        build.build()
    return dfr.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_list():
    assert declared_functions() == sorted(dfr.EXPORTED)


def test_every_declared_symbol_is_exported(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_every_option_is_documented():
    """The option names dfr_set_option accepts are exactly those include/dfr.h lists."""
    src = open(os.path.join(ROOT, "paper_2207_14334_amd", "csrc", "dfr.cpp")).read()
    a = src.index("dfr_status dfr_set_option(")
    body = src[a:src.index("\n}\n", a)]
    accepted = set(re.findall(r'strcmp\(name, "([a-z_]+)"\)', body))
    documented = set(re.findall(r'^ \*   "([a-z_]+)"', open(HEADER).read(), flags=re.M))
    assert accepted and accepted == documented, (accepted ^ documented)


def test_temp_bytes(L):
    assert dfr.temp_bytes(0, 4, 0) == 0
    assert dfr.temp_bytes(1, 4, 0) == 256
    assert dfr.temp_bytes(1 << 20, 4, 4) == (1 << 23)
    assert dfr.temp_bytes(1000, 8, 8) == 8192 + 8192
    assert dfr.temp_bytes(10, 3, 0) == 0  # bad width


def test_local_sort_capacity(L):
    assert dfr.local_sort_capacity(4, 0) == 8192
    assert dfr.local_sort_capacity(4, 4) == 8192
    assert dfr.local_sort_capacity(8, 8) == 4096
    assert dfr.local_sort_capacity(5, 0) == 0


def test_status_strings(L):
    for st in range(-9, 1):
        assert dfr.status_string(st)
    assert dfr.status_string(0) == "ok"


def test_null_context_and_bad_arguments(L):
    P = ctypes.c_void_p
    assert L.dfr_sort_u32(None, P(4096), None, 10, None, 0, None) == dfr.E_INVALID_ARG
    assert L.dfr_sort_u64(None, None, None, 0, None, 0, None) == dfr.E_INVALID_ARG
    assert L.dfr_set_option(None, b"timing", 1) == dfr.E_INVALID_ARG
    assert L.dfr_get_stats(None, None) == dfr.E_INVALID_ARG
    out = P()
    assert L.dfr_create(0, 0, None) == dfr.E_INVALID_ARG
    assert L.dfr_count(None, None, 4, 0, 8, 4, None, None) == dfr.E_INVALID_ARG
    off = (ctypes.c_uint64 * 3)(0, 5, 3)  # decreasing offsets
    assert L.dfr_sort_segmented_u32(None, P(4096), None, off, 2, None, 0, None) == dfr.E_INVALID_ARG
    t = ctypes.c_uint64(0)
    req = dfr.Request(4, 4, 4096, 8192, 10)
    assert L.dfr_submit(None, ctypes.byref(req), ctypes.byref(t)) == dfr.E_INVALID_ARG
    assert L.dfr_poll(None, 1, None) == dfr.E_INVALID_ARG
    assert L.dfr_get_serve_stats(None, None) == dfr.E_INVALID_ARG
    assert L.dfr_autotune(None, 4, 4, None, None, None, 0, 1, None, None) == dfr.E_INVALID_ARG
    assert L.dfr_get_tune(None, 4, 4, 0, None) == dfr.E_INVALID_ARG
    assert L.dfr_set_tune(None, 4, 4, 0, None) == dfr.E_INVALID_ARG
    assert L.dfr_stream_copy(None, P(4096), P(8192), 16, None) == dfr.E_INVALID_ARG
    assert L.dfr_stream_read(None, P(4096), 16, P(8192), None) == dfr.E_INVALID_ARG


def test_create_without_gpu_fails_cleanly(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    out = ctypes.c_void_p()
    assert L.dfr_create(0, 0, ctypes.byref(out)) == dfr.E_HIP
    assert not out.value


# --------------------------------------------------------------------------------------
# Planner (Sec. 3: estimate the top digits to deal; Sec. 3.1: threshold N_d).
# --------------------------------------------------------------------------------------

def hist_of(keys, kb):
    h = np.zeros((kb, 256), dtype=np.uint32)
    for j in range(kb):
        d = ((keys >> keys.dtype.type(8 * j)) & keys.dtype.type(255)).astype(np.int64)
        h[j] = np.bincount(d, minlength=256)
    return h


def uniform_hist(n, kb):
    return np.full((kb, 256), n // 256, dtype=np.uint32)


def test_plan_uniform_u32_2p28(L):
    # Expected bucket after d top digits: 2^28 / 256^d; N_d = 6144 -> d = 2.
    d, v = dfr.plan_top_digits(uniform_hist(1 << 28, 4), 1 << 28, 4, 4)
    assert (d, v) == (2, 4)


def test_plan_uniform_u64_2p27(L):
    # 2^27 / 256^2 = 2048 <= N_d = 3072 for 16-byte records -> d = 2.
    d, v = dfr.plan_top_digits(uniform_hist(1 << 27, 8), 1 << 27, 8, 8)
    assert (d, v) == (2, 8)


def test_plan_small_input_diverts_at_once(L):
    d, _ = dfr.plan_top_digits(uniform_hist(8192, 4), 8192, 4, 4)
    assert d == 0


def test_plan_skips_constant_digits(L):
    k = workloads.make_keys("narrow", 1 << 20, 32, 0, narrow_bits=20)
    d, v = dfr.plan_top_digits(hist_of(k, 4), k.size, 4, 0)
    assert v == 3  # bits 20..31 are zero: digit 3 never varies
    assert 1 <= d <= 3


def test_plan_all_equal(L):
    k = workloads.make_keys("equal", 1 << 16, 64, 0)
    d, v = dfr.plan_top_digits(hist_of(k, 8), k.size, 8, 8)
    assert v == 0 and d == 0


def test_plan_skewed_prefers_full_lsd(L):
    # Zipf keys: most records share their top digits, so no short prefix reaches N_d
    # and dealing every digit moves the fewest bytes.
    k = workloads.make_keys("zipf", 1 << 20, 32, 0)
    h = hist_of(k, 4) * 256  # as if n were 2^28 with the same shape
    d, v = dfr.plan_top_digits(h, 1 << 28, 4, 4)
    assert d == v == 4


def test_plan_divert_option_changes_depth(L):
    h = uniform_hist(1 << 28, 4)
    assert dfr.plan_top_digits(h, 1 << 28, 4, 4, divert=64)[0] == 4  # LSD is cheaper
    assert dfr.plan_top_digits(h + np.uint32(3) * (np.arange(256) % 2).astype(np.uint32), 1 << 28, 4, 4)[0] == 2
    assert dfr.plan_top_digits(h, 1 << 28, 4, 4, divert=8192)[0] == 2


def test_deal_tile_records(L):
    assert dfr.deal_tile_records(4, 4) == 8192
    assert dfr.deal_tile_records(4, 0) == 8192
    assert dfr.deal_tile_records(8, 8) == 4096
    assert dfr.deal_tile_records(3, 4) == 0


def test_size_class_is_log2_of_size_biased_mean():
    # One segment: floor(log2 n).
    assert dfr.size_class([0, 1 << 20]) == 20
    assert dfr.size_class([0, (1 << 20) - 1]) == 19
    # Segments of one record or none do not count; the mean is weighted by length:
    # lengths 1000 and 3000 give (1000^2 + 3000^2) / 4000 = 2500 -> 11.
    assert dfr.size_class([0, 0, 1, 1001, 4001]) == 11
    # Nothing to sort -> class 0.
    assert dfr.size_class([0, 1, 2]) == 0
    with pytest.raises(dfr.DfrError):
        dfr.size_class([5, 10])
    with pytest.raises(dfr.DfrError):
        dfr.size_class([0, 10, 5])


def test_size_limit_macro_in_expressions(tmp_path):
    """DFR_MAX_SEGMENT_RECORDS is one parenthesised value (2^32 - 1): it can be used in
    any C expression."""
    import subprocess
    src = tmp_path / "limit.c"
    src.write_text(
        '#include <stdio.h>\n#include "dfr.h"\n'
        "int main(void) {\n"
        "    size_t x = (size_t)1 << 33;\n"
        '    printf("%zu %zu %zu\\n", (size_t)(2 * DFR_MAX_SEGMENT_RECORDS),\n'
        "           (size_t)(x % DFR_MAX_SEGMENT_RECORDS), (size_t)(~DFR_MAX_SEGMENT_RECORDS >> 32));\n"
        "    return 0;\n}\n")
    exe = tmp_path / "limit"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    m = (1 << 32) - 1
    assert [int(v) for v in out] == [2 * m, (1 << 33) % m, ((~m) & ((1 << 64) - 1)) >> 32]
    assert dfr.MAX_SEGMENT_RECORDS == m
