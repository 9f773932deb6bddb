"""Seeded synthetic columns for tests and benchmarks (inputs only).

A thin ctypes wrapper over ``datagen.c``.  It produces data and holds none of
the aggregation arithmetic, so both the GPU library's tests and the CPU oracle
take their inputs from here without sharing any of the method.

Every column is a pure function of ``(dtype, dist, n, seed, lo, hi)`` and is
identical whatever thread count produced it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "datagen.c")
_LIB = os.path.join(_HERE, "libdatagen.so")

I32, I64, F32 = 0, 1, 2
UNIFORM, ZIPF, SORTED, NORMAL_OUTLIERS = 0, 1, 2, 3

DTYPES = {"i32": I32, "i64": I64, "f32": F32}
DISTS = {"uniform": UNIFORM, "zipf": ZIPF, "sorted": SORTED,
         "normal_outliers": NORMAL_OUTLIERS}
NP_DTYPE = {I32: np.int32, I64: np.int64, F32: np.float32}
WIDTH = {I32: 4, I64: 8, F32: 4}

_lib = None


def build() -> str:
    """Compile the generator library with gcc (always recompiles)."""
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
        lib.dg_fill.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
        lib.dg_fill.restype = ctypes.c_int
        lib.dg_raw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.dg_raw.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def default_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return min(16, os.cpu_count() or 1)


def _code(v, table):
    return table[v] if isinstance(v, str) else int(v)


def fill_ptr(ptr: int, n: int, dtype, dist, seed: int, lo: int = 0, hi: int = 0,
             threads: int | None = None) -> None:
    """Write the column into host memory at ``ptr`` (e.g. a pinned tensor)."""
    rc = _load().dg_fill(ctypes.c_void_p(ptr), n, _code(dtype, DTYPES), _code(dist, DISTS),
                         seed, lo, hi, threads or default_threads())
    if rc != 0:
        raise ValueError(f"dg_fill failed rc={rc} (dtype={dtype} dist={dist} n={n})")


def column(n: int, dtype="i32", dist="uniform", seed: int = 1, lo: int = 0, hi: int = 0,
           threads: int | None = None) -> np.ndarray:
    """Return a new numpy column."""
    dt = _code(dtype, DTYPES)
    out = np.empty(n, dtype=NP_DTYPE[dt])
    if n:
        fill_ptr(out.ctypes.data, n, dt, dist, seed, lo, hi, threads)
    return out


def raw(seed: int, ctr: int) -> int:
    """Raw 64-bit output ``ctr`` of the generator's first stream for ``seed``."""
    return int(_load().dg_raw(seed, ctr))


# Reference SplitMix64 in plain Python, for the generator's own tests.
_M64 = (1 << 64) - 1


def splitmix64_mix(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)
