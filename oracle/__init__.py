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
