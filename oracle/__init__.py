"""CPU oracle for the Diverting Fast Radix (DFR) sort (arXiv 2207.14334).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library and its
Python binding never touch it, and it shares no code with them.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc into ``liboracle.so``);
this module only marshals numpy arrays.  What each function computes, and the passage
of the paper it follows, is stated in ``oracle.c``:

* ``stable_sort`` -- the definition of the result: record i goes to
  rank(i) = #{j: k_j < k_i} + #{j < i: k_j == k_i}  (Sec. 2.1 stability, Sec. 3).
* ``stable_sort_parallel`` -- the same result on several host threads (chunks sorted
  by that definition, then merged pairwise with equal keys left first), for timing.
* ``rank`` -- that formula evaluated directly, O(n^2).
* ``count`` / ``deal`` -- one counting-sort pass (Sec. 2, counting sort paragraph).
* ``lsd_sort`` -- LSD radix sort from the deals (Sec. 2.1).
* ``dfr_sort`` -- DFR's steps in the order Sec. 3 gives them.
* ``bucket_starts`` -- where the leading-digit prefix changes (Sec. 2.2 buckets).
* ``check_index_payload`` -- the four properties that single out the stable sort
  when the payload is the input index.
* ``stable_sort_typed`` -- the stable sort of signed-integer or floating-point keys
  (two's-complement value; IEEE 754 totalOrder), beyond the paper's unsigned keys.
* ``overflow_fraction`` -- Eq. 2, the expected overflow of Fast Radix's estimated buckets.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_KB = {np.dtype(np.uint32): 4, np.dtype(np.uint64): 8}


def build(out_path: str = _LIB, defines: tuple[str, ...] = ()) -> str:
    """Compile oracle.c with gcc into a shared library at ``out_path``.

    ``defines`` are preprocessor symbols; the pin tests use them to build copies of
    the oracle with a planted mistake and check that the pins catch it.
    """
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", _SRC, "-o",
           out_path + ".tmp", "-lm", "-lpthread"]
    cmd[1:1] = [f"-D{d}" for d in defines]
    subprocess.run(cmd, check=True)
    os.replace(out_path + ".tmp", out_path)
    return out_path


class Oracle:
    """numpy front end of one build of liboracle.so."""

    def __init__(self, path: str = _LIB):
        if not os.path.exists(path):
            build(path)
        self.path = path
        lib = ctypes.CDLL(path)
        P, Z, I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        lib.oracle_stable_sort.argtypes = [P, P, Z, I, I, P, P]
        lib.oracle_stable_sort_parallel.argtypes = [P, P, Z, I, I, I, P, P]
        lib.oracle_segmented_sort.argtypes = [P, P, Z, I, I, P, Z, P, P]
        lib.oracle_rank.argtypes = [P, Z, I, P]
        lib.oracle_rank_of.argtypes = [P, Z, I, Z]
        lib.oracle_rank_of.restype = ctypes.c_uint64
        lib.oracle_count.argtypes = [P, Z, I, I, I, P]
        lib.oracle_deal.argtypes = [P, P, Z, I, I, I, I, P, P]
        lib.oracle_lsd_sort.argtypes = [P, P, Z, I, I, I, P, P]
        lib.oracle_bucket_starts.argtypes = [P, Z, I, I, P, Z]
        lib.oracle_bucket_starts.restype = ctypes.c_size_t
        lib.oracle_dfr_sort.argtypes = [P, P, Z, I, I, I, Z, P, P]
        lib.oracle_check_index_payload.argtypes = [P, Z, I, P, P, I, ctypes.POINTER(I)]
        lib.oracle_check_index_payload.restype = ctypes.c_int64
        lib.oracle_stable_sort_typed.argtypes = [P, P, Z, I, I, P, P]
        lib.oracle_overflow_fraction.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
        lib.oracle_overflow_fraction.restype = ctypes.c_double
        self.lib = lib

    # -- helpers ---------------------------------------------------------------
    @staticmethod
    def _prep(keys, vals):
        keys = np.ascontiguousarray(keys)
        if keys.dtype not in _KB:
            raise TypeError("keys must be uint32 or uint64")
        kb = _KB[keys.dtype]
        if vals is None:
            return keys, None, kb, 0
        vals = np.ascontiguousarray(vals)
        if vals.dtype not in _KB or vals.shape != keys.shape:
            raise TypeError("vals must be uint32/uint64 and match keys")
        return keys, vals, kb, _KB[vals.dtype]

    @staticmethod
    def _p(a):
        return None if a is None else a.ctypes.data

    @staticmethod
    def _rc(rc):
        if rc != 0:
            raise RuntimeError(f"oracle returned {rc}")

    # -- the definition ----------------------------------------------------------
    def stable_sort(self, keys, vals=None):
        keys, vals, kb, vb = self._prep(keys, vals)
        ok = np.empty_like(keys)
        ov = np.empty_like(vals) if vals is not None else None
        self._rc(self.lib.oracle_stable_sort(self._p(keys), self._p(vals), keys.size, kb, vb,
                                             self._p(ok), self._p(ov)))
        return ok, ov

    def stable_sort_parallel(self, keys, vals=None, threads: int = 1):
        keys, vals, kb, vb = self._prep(keys, vals)
        ok = np.empty_like(keys)
        ov = np.empty_like(vals) if vals is not None else None
        self._rc(self.lib.oracle_stable_sort_parallel(self._p(keys), self._p(vals), keys.size,
                                                      kb, vb, int(threads), self._p(ok),
                                                      self._p(ov)))
        return ok, ov

    def overflow_fraction(self, N: int, M: int) -> float:
        """Eq. 2: expected overflow of N uniform records dealt into M buckets of N/M slots,
        as a fraction of N (Sec. 3.1)."""
        return float(self.lib.oracle_overflow_fraction(N, M))

    # Key types of stable_sort_typed, by numpy dtype of the keys.
    KEY_TYPES = {np.dtype(np.uint32): 0, np.dtype(np.uint64): 1, np.dtype(np.int32): 2,
                 np.dtype(np.int64): 3, np.dtype(np.float32): 4, np.dtype(np.float64): 5}

    def stable_sort_typed(self, keys, vals=None):
        """Stable sort of uint/int/float keys (their raw encodings are sorted under the
        type's order and returned unchanged)."""
        keys = np.ascontiguousarray(keys)
        kt = self.KEY_TYPES[keys.dtype]
        vb = 0
        if vals is not None:
            vals = np.ascontiguousarray(vals)
            if vals.dtype not in _KB or vals.shape != keys.shape:
                raise TypeError("vals must be uint32/uint64 and match keys")
            vb = _KB[vals.dtype]
        ok = np.empty_like(keys)
        ov = np.empty_like(vals) if vals is not None else None
        self._rc(self.lib.oracle_stable_sort_typed(self._p(keys), self._p(vals), keys.size, kt, vb,
                                                   self._p(ok), self._p(ov)))
        return ok, ov

    def segmented_sort(self, keys, vals, offsets):
        keys, vals, kb, vb = self._prep(keys, vals)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        ok = np.empty_like(keys)
        ov = np.empty_like(vals) if vals is not None else None
        self._rc(self.lib.oracle_segmented_sort(self._p(keys), self._p(vals), keys.size, kb, vb,
                                                off.ctypes.data, off.size - 1, self._p(ok),
                                                self._p(ov)))
        return ok, ov

    def rank(self, keys):
        keys, _, kb, _ = self._prep(keys, None)
        r = np.empty(keys.size, dtype=np.uint64)
        self._rc(self.lib.oracle_rank(self._p(keys), keys.size, kb, r.ctypes.data))
        return r

    def rank_of(self, keys, i):
        keys, _, kb, _ = self._prep(keys, None)
        return int(self.lib.oracle_rank_of(self._p(keys), keys.size, kb, int(i)))

    # -- stages ------------------------------------------------------------------
    def count(self, keys, shift, bits):
        keys, _, kb, _ = self._prep(keys, None)
        h = np.empty(1 << bits, dtype=np.uint64)
        self._rc(self.lib.oracle_count(self._p(keys), keys.size, kb, shift, bits, h.ctypes.data))
        return h

    def deal(self, keys, vals, shift, bits):
        keys, vals, kb, vb = self._prep(keys, vals)
        ok = np.empty_like(keys)
        ov = np.empty_like(vals) if vals is not None else None
        self._rc(self.lib.oracle_deal(self._p(keys), self._p(vals), keys.size, kb, vb, shift,
                                      bits, self._p(ok), self._p(ov)))
        return ok, ov

    def lsd_sort(self, keys, vals=None, bits=8):
        keys, vals, kb, vb = self._prep(keys, vals)
        ok = np.empty_like(keys)
        ov = np.empty_like(vals) if vals is not None else None
        self._rc(self.lib.oracle_lsd_sort(self._p(keys), self._p(vals), keys.size, kb, vb, bits,
                                          self._p(ok), self._p(ov)))
        return ok, ov

    def dfr_sort(self, keys, vals=None, bits=8, divert=64):
        keys, vals, kb, vb = self._prep(keys, vals)
        ok = np.empty_like(keys)
        ov = np.empty_like(vals) if vals is not None else None
        self._rc(self.lib.oracle_dfr_sort(self._p(keys), self._p(vals), keys.size, kb, vb, bits,
                                          divert, self._p(ok), self._p(ov)))
        return ok, ov

    def bucket_starts(self, keys, lo_bit):
        keys, _, kb, _ = self._prep(keys, None)
        c = self.lib.oracle_bucket_starts(self._p(keys), keys.size, kb, lo_bit, None, 0)
        s = np.empty(max(c, 1), dtype=np.uint64)
        self.lib.oracle_bucket_starts(self._p(keys), keys.size, kb, lo_bit, s.ctypes.data, c)
        return s[:c]

    def check_index_payload(self, in_keys, out_keys, out_vals):
        """Return None when the four properties hold, else (position, property)."""
        in_keys = np.ascontiguousarray(in_keys)
        out_keys = np.ascontiguousarray(out_keys)
        out_vals = np.ascontiguousarray(out_vals)
        if out_keys.dtype != in_keys.dtype or out_keys.shape != in_keys.shape:
            return (0, 0)
        what = ctypes.c_int(0)
        p = self.lib.oracle_check_index_payload(in_keys.ctypes.data, in_keys.size,
                                                _KB[in_keys.dtype], out_keys.ctypes.data,
                                                out_vals.ctypes.data, _KB[out_vals.dtype],
                                                ctypes.byref(what))
        return None if p < 0 else (int(p), int(what.value))


_default: Oracle | None = None


def get() -> Oracle:
    """The oracle built from the unmodified source."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
