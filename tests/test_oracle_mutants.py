"""The oracle's pins are strong enough to catch plausible mistakes.

Each case copies ``oracle/oracle.c``, plants one mistake (a dropped term, a
wrong sign or index, a narrowed accumulator, a wrong rounding rule), builds the
copy into a temporary library on the CPU, and checks that at least one of the
pin checks below fails for it, while all of them pass for the real oracle.
"""
import ctypes
import math
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "exponent_off_by_one": ("k = (int)biased - 1;", "k = (int)biased;"),
    "high_digit_sign_dropped": ("{ lo = -lo; hi = -hi; }", "{ lo = -lo; }"),
    "high_digit_dropped": ("a->d[k / 32 + 1] += hi;", "(void)hi;"),
    "round_half_up": ("if (round && (sticky || (mant & 1)))", "if (round)"),
    "sticky_ignored": ("if (round && (sticky || (mant & 1)))", "if (round && (mant & 1))"),
    "truncate_not_round": ("if (round && (sticky || (mant & 1))) {", "if (0) {"),
    "narrow_int_accumulator": ("j->wrap_sum += (uint64_t)x;", "j->wrap_sum = (uint32_t)(j->wrap_sum + (uint64_t)x);"),
    "last_item_dropped": ("for (int64_t i = j->lo; i < j->hi; ++i)", "for (int64_t i = j->lo; i + 1 < j->hi; ++i)"),
    "range_overlap": ("jobs[t].lo = n * t / nt;", "jobs[t].lo = t ? n * t / nt - 1 : 0;"),
    "min_compare_flipped": ("if (x < j->imin) j->imin = x;", "if (x > j->imin) j->imin = x;"),
    "fmax_compare_flipped": ("(isnan(j->fmax) || x > j->fmax)", "(isnan(j->fmax) || x < j->fmax)"),
    "avg_integer_division": ("out->f64 = (double)s / (double)n;", "out->f64 = (double)(s / n);"),
    "negative_sum_not_renormalised": ("d[k] -= carry * 4294967296LL;\n            d[k + 1] += carry;\n        }\n    }",
                                      "(void)carry;\n        }\n    }"),
    "merge_skips_thread": ("if (dtype == O_F32) sa_merge(&m->sa, &jobs[t].sa);",
                           "if (dtype == O_F32 && t != 1) sa_merge(&m->sa, &jobs[t].sa);"),
    "groupby_run_cut_short": ("for (; j < n && key_at(keys, key_dtype, idx[j]) == k; ++j) {",
                              "for (; j < n && (j == i || key_at(keys, key_dtype, idx[j - 1]) == k) && key_at(keys, key_dtype, idx[j]) == k && j - i < 5; ++j) {"),
    "groupby_compare_flipped": ("return (ka > kb) - (ka < kb);", "return (ka < kb) - (ka > kb);"),
    "groupby_count_off": ("g->count = j - i;", "g->count = j - i + (j == n);"),
}


class _Res(ctypes.Structure):
    _fields_ = [("i64", ctypes.c_int64), ("f64", ctypes.c_double), ("count", ctypes.c_int64),
                ("is_null", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Grp(ctypes.Structure):
    _fields_ = [("key", ctypes.c_int64), ("i64", ctypes.c_int64), ("f64", ctypes.c_double),
                ("count", ctypes.c_int64)]


def _build(src_text: str, path: str):
    c = path + ".c"
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-w", "-ffp-contract=off", "-fPIC",
                           "-shared", "-pthread", "-o", path, c, "-lm"])
    lib = ctypes.CDLL(path)
    lib.oracle_aggregate.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.POINTER(_Res)]
    lib.oracle_groupby.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                   ctypes.c_int, ctypes.POINTER(_Grp), ctypes.c_int64]
    lib.oracle_groupby.restype = ctypes.c_int64
    return lib


def _agg(lib, x: np.ndarray, op: int, threads: int = 4):
    dt = {np.dtype(np.int32): 0, np.dtype(np.int64): 1, np.dtype(np.float32): 2}[x.dtype]
    r = _Res()
    rc = lib.oracle_aggregate(ctypes.c_void_p(x.ctypes.data), x.size, dt, op, threads, ctypes.byref(r))
    assert rc == 0
    return r


def _cr(fr: Fraction) -> float:
    return fr.numerator / fr.denominator


def _pin_failures(lib) -> list:
    """Run a compact set of the oracle's pins; return the names that fail."""
    bad = []
    r = np.random.default_rng(1)
    xi = r.integers(-2**31, 2**31, size=200_003, dtype=np.int32)
    if _agg(lib, xi, 0).i64 != int(xi.astype(np.int64).sum()):
        bad.append("int_sum")
    if _agg(lib, xi, 1).i64 != int(xi.min()) or _agg(lib, xi, 2).i64 != int(xi.max()):
        bad.append("int_minmax")
    if _agg(lib, np.full(5, -2**31, np.int32), 0, 1).i64 != -5 * 2**31:
        bad.append("int_widen")
    a = np.arange(7, dtype=np.int64)
    if _agg(lib, a, 4, 1).f64 != 3.0 or _agg(lib, np.array([1, 2], np.int64), 4, 1).f64 != 1.5:
        bad.append("avg")
    xf = (r.standard_normal(3000) * np.exp2(r.integers(-40, 41, size=3000))).astype(np.float32)
    exact = sum((Fraction(float(v)) for v in xf), Fraction(0))
    if _agg(lib, xf, 0, 1).f64 != _cr(exact):
        bad.append("f32_sum_exact")
    big = r.standard_normal(300_007).astype(np.float32)
    if _agg(lib, big, 0, 4).f64 != math.fsum(big.astype(np.float64).tolist()):
        bad.append("f32_sum_fsum_threads")
    if _agg(lib, -np.abs(xf), 0, 1).f64 != _cr(-sum((Fraction(abs(float(v))) for v in xf), Fraction(0))):
        bad.append("f32_negative_sum")
    t = np.float32(2.0**53)
    if _agg(lib, np.array([t, 1.0], np.float32), 0, 1).f64 != 2.0**53:
        bad.append("tie_even")
    if _agg(lib, np.array([t, 1.0, 2.0**-20], np.float32), 0, 1).f64 != 2.0**53 + 2:
        bad.append("sticky")
    if _agg(lib, np.array([t, 3.0], np.float32), 0, 1).f64 != 2.0**53 + 4:
        bad.append("round_up")
    if _agg(lib, big, 2, 4).f64 != float(big.max()) or _agg(lib, big, 1, 4).f64 != float(big.min()):
        bad.append("f32_minmax")
    # group-by: against a Python dict
    gk = r.integers(-50, 50, size=5000).astype(np.int64)
    gv = r.integers(-1000, 1000, size=5000).astype(np.int32)
    out = (_Grp * 200)()
    ng = lib.oracle_groupby(gk.ctypes.data, 1, gv.ctypes.data, 0, gk.size, 0, out, 200)
    want = {}
    for k, v in zip(gk.tolist(), gv.tolist()):
        want[k] = want.get(k, 0) + v
    cnt = {k: int((gk == k).sum()) for k in want}
    got = [(out[i].key, out[i].i64, out[i].count) for i in range(min(ng, 200))]
    if ng != len(want) or got != [(k, want[k], cnt[k]) for k in sorted(want)]:
        bad.append("groupby")
    return bad


def test_real_oracle_passes_every_pin(tmp_path):
    lib = _build(open(SRC).read(), str(tmp_path / "real.so"))
    assert _pin_failures(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    lib = _build(src.replace(old, new, 1), str(tmp_path / f"{name}.so"))
    assert _pin_failures(lib), f"no pin caught the planted mistake {name}"
