"""Python binding of libdfr.so: a GPU Diverting Fast Radix sort for MI355X (gfx950).

This module only marshals arguments: every step of the sort runs in the HIP kernels of
``libdfr.so`` (see ``include/dfr.h`` for the C ABI).  PyTorch provides the device memory
and the stream; tensors must live on a ROCm device, be contiguous and have dtype
``torch.uint32`` or ``torch.uint64``.

If ``libdfr.so`` has not been built, importing works but every GPU entry point raises
``RuntimeError``: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfr.so")

# Status codes (include/dfr.h).
OK = 0
E_INVALID_ARG = -1
E_TOO_LARGE = -2
E_NO_MEMORY = -3
E_HIP = -4
E_PENDING = -5
E_NOT_FOUND = -6
E_BUDGET = -7
E_UNSUPPORTED = -8
E_INTERNAL = -9

MAX_SEGMENT_RECORDS = (1 << 32) - 1

EXPORTED = [
    "dfr_create", "dfr_destroy", "dfr_status_string", "dfr_last_error", "dfr_temp_bytes",
    "dfr_sort_u32", "dfr_sort_u64", "dfr_sort_segmented_u32", "dfr_sort_segmented_u64",
    "dfr_count", "dfr_deal", "dfr_submit", "dfr_poll", "dfr_set_option", "dfr_get_stats",
    "dfr_plan_top_digits", "dfr_local_sort_capacity", "dfr_deal_tile_records",
    "dfr_size_class", "dfr_autotune", "dfr_get_tune", "dfr_set_tune", "dfr_get_serve_stats",
    "dfr_sort_keys", "dfr_sort_segmented_keys", "dfr_sort_noalloc", "dfr_stream_copy",
    "dfr_stream_read",
]

# The allocation-free entry point's limits (include/dfr.h).
NOALLOC_MAX_RECORDS = 1 << 22
NOALLOC_SCRATCH_BYTES = 192 << 20

# Key types of dfr_sort_keys.
KEY_U32, KEY_U64, KEY_I32, KEY_I64, KEY_F32, KEY_F64 = range(6)

TUNE_CLASSES = 32


class DfrError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"dfr status {status}: {msg}")


class Stats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("top_digits", ctypes.c_int32),
        ("deal_passes", ctypes.c_int32), ("used_diversion", ctypes.c_int32),
        ("large_buckets", ctypes.c_uint64), ("chunks", ctypes.c_uint64),
        ("ms_count", ctypes.c_double), ("ms_deal", ctypes.c_double),
        ("ms_buckets", ctypes.c_double), ("ms_local_sort", ctypes.c_double),
        ("ms_other", ctypes.c_double), ("deal_launches_timed", ctypes.c_int32),
        ("estimated_overflow", ctypes.c_double),
        ("chunks_form0", ctypes.c_uint64), ("chunks_form1", ctypes.c_uint64),
        ("chunks_form2", ctypes.c_uint64), ("chunks_general", ctypes.c_uint64),
        ("deal_passes_scanned", ctypes.c_int32), ("deal_passes_lookback", ctypes.c_int32),
        ("levels_heads_keys", ctypes.c_int32), ("levels_heads_counts", ctypes.c_int32),
        ("levels_heads_hist", ctypes.c_int32), ("deal_passes_estimated", ctypes.c_int32),
        ("plan_from_lengths", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tune(ctypes.Structure):
    _fields_ = [("radix_bits", ctypes.c_int32), ("tile_records", ctypes.c_uint32),
                ("divert_records", ctypes.c_uint64), ("window_records", ctypes.c_uint64),
                ("ms", ctypes.c_double), ("ms_default", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        return cls(**{f: d.get(f, 0) for f, _ in cls._fields_})


class ServeStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("requests", ctypes.c_uint64),
                ("records", ctypes.c_uint64), ("max_batch_requests", ctypes.c_uint64),
                ("peak_held_bytes", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64),
                ("held_bytes", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("allocs", ctypes.c_uint64), ("ms_alloc", ctypes.c_double),
                ("ms_batch_wall", ctypes.c_double), ("ms_gather", ctypes.c_double),
                ("ms_sort", ctypes.c_double), ("ms_scatter", ctypes.c_double),
                ("workers", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [("key_bytes", ctypes.c_int), ("val_bytes", ctypes.c_int),
                ("keys", ctypes.c_void_p), ("vals", ctypes.c_void_p), ("n", ctypes.c_size_t)]


_lib = None


def lib():
    """The loaded libdfr.so.  Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "or python -m paper_2207_14334_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, Z, I, S = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int32
    L.dfr_create.argtypes = [I, Z, ctypes.POINTER(P)]
    L.dfr_create.restype = S
    L.dfr_destroy.argtypes = [P]
    L.dfr_destroy.restype = None
    L.dfr_status_string.argtypes = [S]
    L.dfr_status_string.restype = ctypes.c_char_p
    L.dfr_last_error.argtypes = [P]
    L.dfr_last_error.restype = ctypes.c_char_p
    L.dfr_temp_bytes.argtypes = [Z, I, I]
    L.dfr_temp_bytes.restype = Z
    L.dfr_local_sort_capacity.argtypes = [I, I]
    L.dfr_local_sort_capacity.restype = Z
    for name in ("dfr_sort_u32", "dfr_sort_u64"):
        f = getattr(L, name)
        f.argtypes = [P, P, P, Z, P, Z, P]
        f.restype = S
    for name in ("dfr_sort_segmented_u32", "dfr_sort_segmented_u64"):
        f = getattr(L, name)
        f.argtypes = [P, P, P, P, Z, P, Z, P]
        f.restype = S
    L.dfr_count.argtypes = [P, P, I, Z, I, I, P, P]
    L.dfr_count.restype = S
    L.dfr_deal.argtypes = [P, P, P, P, P, I, I, Z, I, I, P]
    L.dfr_deal.restype = S
    L.dfr_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.dfr_submit.restype = S
    L.dfr_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
    L.dfr_poll.restype = S
    L.dfr_set_option.argtypes = [P, ctypes.c_char_p, ctypes.c_int64]
    L.dfr_set_option.restype = S
    L.dfr_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.dfr_get_stats.restype = S
    L.dfr_plan_top_digits.argtypes = [P, Z, I, I, Z, ctypes.POINTER(S), ctypes.POINTER(S)]
    L.dfr_plan_top_digits.restype = S
    L.dfr_deal_tile_records.argtypes = [I, I]
    L.dfr_deal_tile_records.restype = Z
    L.dfr_size_class.argtypes = [P, Z]
    L.dfr_size_class.restype = S
    L.dfr_autotune.argtypes = [P, I, I, P, P, P, Z, I, P, ctypes.POINTER(Tune)]
    L.dfr_autotune.restype = S
    L.dfr_get_tune.argtypes = [P, I, I, S, ctypes.POINTER(Tune)]
    L.dfr_get_tune.restype = S
    L.dfr_set_tune.argtypes = [P, I, I, S, ctypes.POINTER(Tune)]
    L.dfr_set_tune.restype = S
    L.dfr_get_serve_stats.argtypes = [P, ctypes.POINTER(ServeStats)]
    L.dfr_get_serve_stats.restype = S
    L.dfr_sort_keys.argtypes = [P, S, P, P, I, Z, P, Z, P]
    L.dfr_sort_keys.restype = S
    L.dfr_sort_segmented_keys.argtypes = [P, S, P, P, I, P, Z, P, Z, P]
    L.dfr_sort_segmented_keys.restype = S
    L.dfr_sort_noalloc.argtypes = [P, P, P, Z, I, I, P]
    L.dfr_sort_noalloc.restype = S
    L.dfr_stream_copy.argtypes = [P, P, P, Z, P]
    L.dfr_stream_copy.restype = S
    L.dfr_stream_read.argtypes = [P, P, Z, P, P]
    L.dfr_stream_read.restype = S
    _lib = L
    return L


def status_string(st: int) -> str:
    return lib().dfr_status_string(st).decode()


def temp_bytes(n: int, key_bytes: int, val_bytes: int) -> int:
    return int(lib().dfr_temp_bytes(n, key_bytes, val_bytes))


def local_sort_capacity(key_bytes: int, val_bytes: int) -> int:
    return int(lib().dfr_local_sort_capacity(key_bytes, val_bytes))


def deal_tile_records(key_bytes: int, val_bytes: int) -> int:
    return int(lib().dfr_deal_tile_records(key_bytes, val_bytes))


def size_class(offsets) -> int:
    """Size class of a segmented call with host ``offsets`` (num_segments + 1 entries)."""
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    c = int(lib().dfr_size_class(off.ctypes.data, off.size - 1))
    if c < 0:
        raise DfrError(E_INVALID_ARG, "size_class: malformed offsets")
    return c


def plan_top_digits(hist, n: int, key_bytes: int, val_bytes: int, divert: int = 0):
    """Host-only planner: (digits dealt before diversion, varying digits) for a
    numpy uint32 histogram array of shape (key_bytes, 256)."""
    import numpy as np
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    d, v = ctypes.c_int32(0), ctypes.c_int32(0)
    st = lib().dfr_plan_top_digits(h.ctypes.data, n, key_bytes, val_bytes, divert,
                                   ctypes.byref(d), ctypes.byref(v))
    if st != OK:
        raise DfrError(st, "plan_top_digits")
    return d.value, v.value


def _width(t) -> int:
    import torch
    if t.dtype in (torch.uint32, torch.int32, torch.float32):
        return 4
    if t.dtype in (torch.uint64, torch.int64, torch.float64):
        return 8
    raise TypeError(f"unsupported dtype {t.dtype}")


def _key_type(t) -> int:
    import torch
    kinds = {torch.uint32: KEY_U32, torch.uint64: KEY_U64, torch.int32: KEY_I32,
             torch.int64: KEY_I64, torch.float32: KEY_F32, torch.float64: KEY_F64}
    if t.dtype not in kinds:
        raise TypeError(f"unsupported key dtype {t.dtype}")
    return kinds[t.dtype]


def _val_width(t) -> int:
    import torch
    if t.dtype in (torch.uint32, torch.int32, torch.float32):
        return 4
    if t.dtype in (torch.uint64, torch.int64, torch.float64):
        return 8
    raise TypeError(f"unsupported value dtype {t.dtype}")


def _check_tensor(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """One libdfr context on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        import torch
        self.device = device
        torch.cuda.set_device(device)
        h = ctypes.c_void_p()
        st = lib().dfr_create(device, hbm_budget_bytes, ctypes.byref(h))
        if st != OK:
            raise DfrError(st, status_string(st))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().dfr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers -------------------------------------------------------------------
    def _raise(self, st, what):
        if st != OK:
            raise DfrError(st, f"{what}: {status_string(st)}: "
                               f"{lib().dfr_last_error(self._h).decode()}")

    @staticmethod
    def _stream(stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        return ctypes.c_void_p(stream.cuda_stream)

    def last_error(self) -> str:
        return lib().dfr_last_error(self._h).decode()

    def set_option(self, name: str, value: int):
        self._raise(lib().dfr_set_option(self._h, name.encode(), int(value)), "set_option")

    def stats(self) -> dict:
        s = Stats()
        self._raise(lib().dfr_get_stats(self._h, ctypes.byref(s)), "get_stats")
        return s.as_dict()

    # -- sorts ---------------------------------------------------------------------
    def sort_(self, keys, vals=None, temp=None, stream=None):
        """Stable in-place ascending sort of ``keys``; ``vals`` follows.  uint32/uint64
        keys sort as unsigned integers (values of the same width), int32/int64 by value,
        float32/float64 by IEEE totalOrder (values 4 or 8 bytes wide, any dtype)."""
        _check_tensor(keys, "keys")
        kt = _key_type(keys)
        n = keys.numel()
        vp, vb = None, 0
        if vals is not None:
            _check_tensor(vals, "vals")
            vb = _val_width(vals)
            if vals.numel() != n:
                raise ValueError("vals must match keys in length")
            vp = vals.data_ptr()
        tp, tb = (temp.data_ptr(), temp.numel() * temp.element_size()) if temp is not None else (None, 0)
        if kt in (KEY_U32, KEY_U64):
            if vals is not None and vb != _width(keys):
                raise ValueError("vals of unsigned keys must match the key width")
            f = lib().dfr_sort_u32 if kt == KEY_U32 else lib().dfr_sort_u64
            self._raise(f(self._h, keys.data_ptr(), vp, n, tp, tb, self._stream(stream)), "sort")
        else:
            self._raise(lib().dfr_sort_keys(self._h, kt, keys.data_ptr(), vp, vb, n, tp, tb,
                                            self._stream(stream)), "sort")
        return keys, vals

    def sort_noalloc_(self, keys, vals=None, stream=None):
        """Stable in-place sort of unsigned ``keys`` (``vals`` follows) that allocates
        no device memory: at most NOALLOC_MAX_RECORDS records, default settings, in the
        library's fixed scratch array on this GPU (calls overlapping on one GPU race)."""
        _check_tensor(keys, "keys")
        if _key_type(keys) not in (KEY_U32, KEY_U64):
            raise TypeError("the allocation-free sort takes uint32 or uint64 keys")
        vp, vb = None, 0
        if vals is not None:
            _check_tensor(vals, "vals")
            if vals.numel() != keys.numel():
                raise ValueError("vals must match keys in length")
            vp, vb = vals.data_ptr(), _val_width(vals)
        self._raise(lib().dfr_sort_noalloc(self._h, keys.data_ptr(), vp, keys.numel(),
                                           _width(keys), vb, self._stream(stream)), "sort_noalloc")
        return keys, vals

    def sort_segmented_(self, keys, vals, offsets, temp=None, stream=None):
        """Sort each segment [offsets[i], offsets[i+1]) of keys/vals independently.
        ``offsets`` holds num_segments + 1 integers: a host sequence, or a contiguous
        uint64/int64 GPU tensor (read back by the library after the queued work)."""
        import numpy as np
        import torch
        _check_tensor(keys, "keys")
        kt = _key_type(keys)
        if isinstance(offsets, torch.Tensor) and offsets.is_cuda:
            if offsets.dtype not in (torch.uint64, torch.int64) or not offsets.is_contiguous():
                raise ValueError("GPU offsets must be a contiguous 64-bit tensor")

            class _DevOffsets:  # the pointer and count the C call needs
                def __init__(self, t):
                    self.ctypes = type("P", (), {"data": t.data_ptr()})()
                    self.size = t.numel()
            off = _DevOffsets(offsets)
        else:
            off = np.ascontiguousarray(offsets, dtype=np.uint64)
        vp, vb = None, 0
        if vals is not None:
            _check_tensor(vals, "vals")
            vp, vb = vals.data_ptr(), _val_width(vals)
        tp, tb = (temp.data_ptr(), temp.numel() * temp.element_size()) if temp is not None else (None, 0)
        if kt in (KEY_U32, KEY_U64) and (vals is None or vb == _width(keys)):
            f = lib().dfr_sort_segmented_u32 if kt == KEY_U32 else lib().dfr_sort_segmented_u64
            self._raise(f(self._h, keys.data_ptr(), vp, off.ctypes.data, off.size - 1, tp, tb,
                          self._stream(stream)), "sort_segmented")
        else:
            self._raise(lib().dfr_sort_segmented_keys(self._h, kt, keys.data_ptr(), vp, vb,
                                                      off.ctypes.data, off.size - 1, tp, tb,
                                                      self._stream(stream)), "sort_segmented")
        return keys, vals

    def stream_copy(self, src, dst, stream=None):
        """Copy GPU tensor ``src`` into ``dst`` (same byte size, a multiple of 16) with
        the library's streaming copy kernel, the bandwidth reference of the passes."""
        _check_tensor(src, "src")
        _check_tensor(dst, "dst")
        nb = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != nb:
            raise ValueError("src and dst must have the same byte size")
        self._raise(lib().dfr_stream_copy(self._h, src.data_ptr(), dst.data_ptr(), nb,
                                          self._stream(stream)), "stream_copy")

    def stream_read(self, src, out, stream=None):
        """Read GPU tensor ``src`` (byte size a multiple of 16) with the library's
        streaming read kernel, the bandwidth reference of the counts, writing the XOR of
        its 32-bit words into ``out`` (a one-element int32/uint32 GPU tensor)."""
        _check_tensor(src, "src")
        _check_tensor(out, "out")
        if out.numel() != 1 or out.element_size() != 4:
            raise ValueError("out must hold one 32-bit word")
        nb = src.numel() * src.element_size()
        self._raise(lib().dfr_stream_read(self._h, src.data_ptr(), nb, out.data_ptr(),
                                          self._stream(stream)), "stream_read")

    # -- tuning --------------------------------------------------------------------
    def autotune(self, keys, vals=None, offsets=None, reps: int = 2, stream=None) -> dict:
        """Tune the launch settings on copies of ``keys``/``vals`` (only read) split by
        host ``offsets`` (None: one segment).  Stores the result in the context and
        returns it as a dict."""
        import numpy as np
        _check_tensor(keys, "keys")
        kb = _width(keys)
        vb, vp = 0, None
        if vals is not None:
            _check_tensor(vals, "vals")
            vb, vp = _width(vals), vals.data_ptr()
        off = np.ascontiguousarray([0, keys.numel()] if offsets is None else offsets, dtype=np.uint64)
        t = Tune()
        self._raise(lib().dfr_autotune(self._h, kb, vb, keys.data_ptr(), vp, off.ctypes.data,
                                       off.size - 1, int(reps), self._stream(stream),
                                       ctypes.byref(t)), "autotune")
        return t.as_dict()

    def get_tune(self, key_bytes: int, val_bytes: int, size_class: int):
        t = Tune()
        st = lib().dfr_get_tune(self._h, key_bytes, val_bytes, size_class, ctypes.byref(t))
        if st == E_NOT_FOUND:
            return None
        self._raise(st, "get_tune")
        return t.as_dict()

    def set_tune(self, key_bytes: int, val_bytes: int, size_class: int, tune):
        t = None if tune is None else ctypes.byref(Tune.from_dict(tune))
        self._raise(lib().dfr_set_tune(self._h, key_bytes, val_bytes, size_class, t), "set_tune")

    def save_tuning(self, path: str):
        """Write every stored setting, with the device's architecture name, as JSON."""
        import json
        import torch
        arch = torch.cuda.get_device_properties(self.device).gcnArchName
        entries = []
        for kb in (4, 8):
            for vb in (0, 4, 8):
                for c in range(TUNE_CLASSES):
                    t = self.get_tune(kb, vb, c)
                    if t is not None:
                        entries.append({"key_bytes": kb, "val_bytes": vb, "size_class": c, **t})
        with open(path, "w") as f:
            json.dump({"arch": arch, "entries": entries}, f, indent=1)

    def load_tuning(self, path: str) -> int:
        """Load settings saved by save_tuning on the same architecture; returns how many."""
        import json
        import torch
        arch = torch.cuda.get_device_properties(self.device).gcnArchName
        with open(path) as f:
            d = json.load(f)
        if d.get("arch") != arch:
            return 0
        for e in d["entries"]:
            self.set_tune(e["key_bytes"], e["val_bytes"], e["size_class"], e)
        return len(d["entries"])

    # -- stages --------------------------------------------------------------------
    def count(self, keys, bits: int = 8, num_digits: int | None = None, stream=None):
        """Digit histograms: returns a (num_digits, 256) uint32 tensor on the device."""
        import torch
        _check_tensor(keys, "keys")
        kb = _width(keys)
        if num_digits is None:
            num_digits = (8 * kb) // bits
        hist = torch.empty((num_digits, 256), dtype=torch.uint32, device=keys.device)
        self._raise(lib().dfr_count(self._h, keys.data_ptr(), kb, keys.numel(), bits, num_digits,
                                    hist.data_ptr(), self._stream(stream)), "count")
        return hist

    def deal(self, keys, vals=None, shift: int = 0, bits: int = 8, stream=None):
        """One stable counting-sort pass on digit (key >> shift) mod 2^bits."""
        import torch
        _check_tensor(keys, "keys")
        kb = _width(keys)
        ko = torch.empty_like(keys)
        vo, vp, vop, vb = None, None, None, 0
        if vals is not None:
            _check_tensor(vals, "vals")
            vb = _width(vals)
            vo = torch.empty_like(vals)
            vp, vop = vals.data_ptr(), vo.data_ptr()
        self._raise(lib().dfr_deal(self._h, keys.data_ptr(), vp, ko.data_ptr(), vop, kb, vb,
                                   keys.numel(), shift, bits, self._stream(stream)), "deal")
        return ko, vo

    # -- request queue -------------------------------------------------------------
    # -- serving -------------------------------------------------------------------
    def submit(self, keys, vals=None) -> int:
        """Queue an in-place sort of ``keys`` (and ``vals``).  The tensors' data must be
        written (e.g. torch.cuda.synchronize()) and must stay alive until poll says done."""
        _check_tensor(keys, "keys")
        kb = _width(keys)
        vb = 0
        if vals is not None:
            _check_tensor(vals, "vals")
            vb = _width(vals)
            if vals.numel() != keys.numel():
                raise ValueError("vals must match keys in length")
        r = Request(kb, vb, keys.data_ptr(), vals.data_ptr() if vals is not None else None,
                    keys.numel())
        t = ctypes.c_uint64(0)
        self._raise(lib().dfr_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "submit")
        return t.value

    def poll(self, ticket: int):
        """(done, latency_seconds or None)."""
        lat = ctypes.c_double(0)
        st = lib().dfr_poll(self._h, ticket, ctypes.byref(lat))
        if st == E_PENDING:
            return False, None
        self._raise(st, "poll")
        return True, lat.value

    def serve_stats(self) -> dict:
        s = ServeStats()
        self._raise(lib().dfr_get_serve_stats(self._h, ctypes.byref(s)), "serve_stats")
        return s.as_dict()


_default_ctx: Context | None = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        import torch
        _default_ctx = Context(torch.cuda.current_device())
    return _default_ctx


def sort_(keys, vals=None, temp=None, stream=None):
    """Stable in-place sort with the default context."""
    return default_context().sort_(keys, vals, temp, stream)


def sort_segmented_(keys, vals, offsets, temp=None, stream=None):
    return default_context().sort_segmented_(keys, vals, offsets, temp, stream)
