"""CPU oracle of the aggregation scan -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU library never imports, links or calls it, and the
two share no code.  ``oracle.c`` states what is computed (Section 2.1 and
Figure 4 of the paper); this module only marshals arguments to it.

Every function here is pinned by ``tests/test_oracle.py`` against brute force
(Python integers, ``fractions.Fraction``, ``math.fsum``), closed forms and
invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

I32, I64, F32 = 0, 1, 2
SUM, MIN, MAX, COUNT, AVG, ABS_SUM = 0, 1, 2, 3, 4, 5
DTYPES = {"i32": I32, "i64": I64, "f32": F32}
OPS = {"sum": SUM, "min": MIN, "max": MAX, "count": COUNT, "avg": AVG, "abs_sum": ABS_SUM}
_NP = {np.dtype(np.int32): I32, np.dtype(np.int64): I64, np.dtype(np.float32): F32}


class _Result(ctypes.Structure):
    _fields_ = [("i64", ctypes.c_int64), ("f64", ctypes.c_double), ("count", ctypes.c_int64),
                ("is_null", ctypes.c_int32), ("reserved", ctypes.c_int32)]


@dataclass
class OracleResult:
    i64: int
    f64: float
    count: int
    is_null: bool

    def value(self, dtype: int, op: int):
        """The natural Python value: int for integer SUM/MIN/MAX and COUNT, else float."""
        if self.is_null:
            return None
        if op == COUNT or (dtype != F32 and op in (SUM, MIN, MAX)):
            return self.i64
        return self.f64


class _Group(ctypes.Structure):
    _fields_ = [("key", ctypes.c_int64), ("i64", ctypes.c_int64), ("f64", ctypes.c_double),
                ("count", ctypes.c_int64)]


_lib = None


def build() -> str:
    """Compile the oracle with gcc (always recompiles).  No fast-math, no FMA contraction."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-ffp-contract=off",
                           "-fno-fast-math", "-fPIC", "-shared", "-pthread",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_aggregate.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Result)]
        lib.oracle_aggregate.restype = ctypes.c_int
        lib.oracle_groupby.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_Group), ctypes.c_int64]
        lib.oracle_groupby.restype = ctypes.c_int64
        lib.oracle_block_aggregate.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_block_aggregate.restype = ctypes.c_int
        lib.oracle_read_ceiling.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_read_ceiling.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return min(16, os.cpu_count() or 1)


def aggregate_ptr(ptr: int, n: int, dtype: int, op: int, threads: int | None = None) -> OracleResult:
    """Aggregate ``n`` items of ``dtype`` at host address ``ptr``."""
    r = _Result()
    rc = _load().oracle_aggregate(ctypes.c_void_p(ptr), n, int(dtype), int(op),
                                  threads or default_threads(), ctypes.byref(r))
    if rc != 0:
        raise ValueError(f"oracle_aggregate rc={rc} (dtype={dtype} op={op} n={n})")
    return OracleResult(int(r.i64), float(r.f64), int(r.count), bool(r.is_null))


def aggregate(col: np.ndarray, op, threads: int | None = None) -> OracleResult:
    """Aggregate a contiguous 1-D numpy column (int32, int64 or float32)."""
    col = np.ascontiguousarray(col)
    dt = _NP.get(col.dtype)
    if dt is None or col.ndim != 1:
        raise TypeError(f"unsupported column {col.dtype} ndim={col.ndim}")
    o = OPS[op] if isinstance(op, str) else int(op)
    return aggregate_ptr(col.ctypes.data if col.size else 0, col.size, dt, o, threads)


def value(col: np.ndarray, op, threads: int | None = None):
    """Convenience: the natural Python value of ``aggregate``."""
    col = np.ascontiguousarray(col)
    o = OPS[op] if isinstance(op, str) else int(op)
    return aggregate(col, o, threads).value(_NP[col.dtype], o)


def error_report(estimate: float, exact: float, abs_sum: float) -> dict:
    """Error of an f32 sum estimate against the exact sum:
    rel = |S^ - S*| / |S*| (None when S* == 0), abs_norm = |S^ - S*| / sum|x|,
    kappa = sum|x| / |S*| (the condition number of the sum)."""
    err = abs(estimate - exact)
    return {
        "rel": (err / abs(exact)) if exact != 0 else None,
        "abs_norm": (err / abs_sum) if abs_sum != 0 else 0.0,
        "kappa": (abs_sum / abs(exact)) if exact != 0 else float("inf"),
    }


def groupby(keys: np.ndarray, vals: np.ndarray, op) -> list:
    """Group-by aggregate: [(key, i64, f64, count)] in ascending key order
    (see oracle_groupby in oracle.c)."""
    keys = np.ascontiguousarray(keys)
    vals = np.ascontiguousarray(vals)
    kd, vd = _NP[keys.dtype], _NP[vals.dtype]
    if kd == F32 or keys.size != vals.size:
        raise TypeError("int32 / int64 keys and values of the same length")
    o = OPS[op] if isinstance(op, str) else int(op)
    n = keys.size
    lib = _load()
    ng = lib.oracle_groupby(keys.ctypes.data if n else None, kd, vals.ctypes.data if n else None, vd, n, o, None, 0)
    if ng < 0:
        raise ValueError(f"oracle_groupby rc={ng}")
    out = (_Group * max(1, ng))()
    ng2 = lib.oracle_groupby(keys.ctypes.data if n else None, kd, vals.ctypes.data if n else None, vd, n, o, out, ng)
    assert ng2 == ng
    return [(out[i].key, out[i].i64, out[i].f64, out[i].count) for i in range(ng)]


def block_table_ptr(ptr: int, n: int, dtype: int, op, block: int, threads: int | None = None) -> np.ndarray:
    """Per-block SUM (mod 2^64) / MIN / MAX of the integer items at host address
    ``ptr``: entry j covers items [j*block, min((j+1)*block, n))."""
    o = OPS[op] if isinstance(op, str) else int(op)
    out = np.empty(max(1, -(-n // block)), dtype=np.int64)
    rc = _load().oracle_block_aggregate(ctypes.c_void_p(ptr), n, int(dtype), o, block, out.ctypes.data,
                                        threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle_block_aggregate rc={rc}")
    return out[: -(-n // block)]


def block_table(col: np.ndarray, op, block: int, threads: int | None = None) -> np.ndarray:
    col = np.ascontiguousarray(col)
    return block_table_ptr(col.ctypes.data if col.size else 0, col.size, _NP[col.dtype], op, block, threads)


class RangeOracle:
    """Exact SUM / MIN / MAX / COUNT / AVG of sub-ranges [off, off + n) of one
    large integer column: whole blocks from the oracle's block tables, the
    partial end blocks from oracle_aggregate on those items.  Results as
    ``aggregate`` returns them."""

    def __init__(self, ptr: int, n: int, dtype: int, block: int = 1 << 16, threads: int | None = None):
        self.ptr, self.n, self.dtype, self.block = ptr, n, int(dtype), block
        self.width = 4 if self.dtype == I32 else 8
        s = block_table_ptr(ptr, n, dtype, SUM, block, threads)
        self.prefix = np.concatenate([np.zeros(1, np.uint64), np.cumsum(s.astype(np.uint64), dtype=np.uint64)])
        self.bmin = block_table_ptr(ptr, n, dtype, MIN, block, threads)
        self.bmax = block_table_ptr(ptr, n, dtype, MAX, block, threads)

    def _part(self, lo: int, hi: int, op: int) -> OracleResult:
        return aggregate_ptr(self.ptr + self.width * lo, hi - lo, self.dtype, op, 1)

    def aggregate(self, off: int, n: int, op) -> OracleResult:
        o = OPS[op] if isinstance(op, str) else int(op)
        if not (0 <= off and off + n <= self.n and n >= 0):
            raise ValueError("range outside the column")
        if o == COUNT or n == 0:
            return aggregate_ptr(self.ptr + self.width * off, n, self.dtype, o, 1)
        lo, hi = off, off + n
        b0, b1 = -(-lo // self.block), hi // self.block      # whole blocks [b0, b1)
        if b0 >= b1:
            return self._part(lo, hi, o)
        parts = [self._part(lo, b0 * self.block, SUM if o == AVG else o) if lo < b0 * self.block else None,
                 self._part(b1 * self.block, hi, SUM if o == AVG else o) if b1 * self.block < hi else None]
        parts = [p for p in parts if p is not None]
        if o in (SUM, AVG):
            s = (int(self.prefix[b1]) - int(self.prefix[b0])) % (1 << 64)
            for p in parts:
                s += p.i64
            s = (s + (1 << 63)) % (1 << 64) - (1 << 63)
            if o == SUM:
                return OracleResult(s, float(s), n, False)
            return OracleResult(0, float(s) / float(n), n, False)
        ext = (min if o == MIN else max)
        v = int(self.bmin[b0:b1].min()) if o == MIN else int(self.bmax[b0:b1].max())
        for p in parts:
            v = ext(v, p.i64)
        return OracleResult(v, float(v), n, False)


def read_ceiling(buf_ptr: int, nbytes: int, threads: int) -> int:
    """Read nbytes of host memory with `threads` threads (the host memory read
    ceiling of the CPU baseline); returns the xor of the words read."""
    x = ctypes.c_uint64()
    rc = _load().oracle_read_ceiling(ctypes.c_void_p(buf_ptr), nbytes, threads, ctypes.byref(x))
    if rc != 0:
        raise ValueError(f"oracle_read_ceiling rc={rc}")
    return int(x.value)
