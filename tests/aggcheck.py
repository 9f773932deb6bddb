"""Shared checks of GPU results against the CPU oracle.

Integer SUM / MIN / MAX / COUNT / AVG and float MIN / MAX must match the oracle
bit for bit.  Float SUM / AVG must lie within the a-priori error bound of the
precision mode for the canonical reduction shape (derivation below); the
compensated mode must in addition be within 1e-6 relative of the exact sum.

Error bounds, with u = 2^-24 (float32) and v = 2^-53 (double), for a column
whose canonical shape has segments of S bytes (m = S / 1024 items per lane
accumulator, 8 butterfly levels inside a wave counting the two component
merges) and nseg segments (k = ceil(nseg / 256) partials folded per lane of the
final combine, then 8 + 2 merge levels), against A = sum |x_i|:

  plain f32     every addition is a float32 rounding whose error is at most
                u times a partial sum bounded by A:
                |err| <= (m + 8 + k + 10) * u * A * (1 + small)
  f64 combine   float32 up to the segment partial, double afterwards:
                |err| <= (m + 8) * u * A + (k + 10) * v * A
  Neumaier      each accumulator's (s, c) pair represents its partial sum with
                error <= 2 m u^2 |partials|; each two-sum merge is exact in s and
                adds one float32 rounding of the correction terms (<= u * 2uA);
                s + c is formed in double (v |S_seg|); then double combine:
                |err| <= (2 m + 2 * 8) * u^2 * A + (k + 12) * v * A
The tests use twice these bounds.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

U32 = 2.0 ** -24
U64 = 2.0 ** -53
REL_GATE_COMPENSATED = 1e-6

DT = {"i32": 0, "i64": 1, "f32": 2}
OPCODE = {"sum": 0, "min": 1, "max": 2, "count": 3, "avg": 4}


def seg_bytes_for(width: int, n: int) -> int:
    """The canonical segment size (restated from the header's rule for the bound only)."""
    total = n * width
    seg = 16 * 1024
    target = -(-total // 8192)
    while seg < target:
        seg <<= 1
    return seg


def float_sum_bound(prec: str, n: int, abs_sum: float) -> float:
    seg = seg_bytes_for(4, n)
    m = seg // 1024
    nseg = -(-(n * 4) // seg) if n else 0
    k = -(-nseg // 256) if nseg else 0
    if prec == "f32":
        b = (m + 8 + k + 10) * U32 * 1.01
    elif prec == "f64_combine":
        b = (m + 8) * U32 * 1.01 + (k + 10) * U64
    else:
        b = (2 * m + 16) * U32 * U32 + (k + 12) * U64
    return 2.0 * b * abs_sum


def check(x: np.ndarray, dtype: str, op: str, prec: str, got: dict, threads=None, ctx="") -> dict:
    """Assert the GPU result `got` (decoded agg_result) against the oracle for column x."""
    n = x.size
    exp = oracle.aggregate(x, OPCODE[op], threads)
    assert got["count"] == n, f"{ctx}: count {got['count']} != {n}"
    if op in ("min", "max", "avg") and n == 0:
        assert got["is_null"], f"{ctx}: empty column must be null"
        return {}
    assert not got["is_null"], f"{ctx}: unexpected null"
    if op == "count":
        assert got["i64"] == n, ctx
        return {}
    if dtype != "f32":
        if op == "avg":
            assert got["f64"] == exp.f64, f"{ctx}: avg {got['f64']!r} != {exp.f64!r}"
        else:
            assert got["i64"] == exp.i64, f"{ctx}: {got['i64']} != {exp.i64}"
        return {}
    if op in ("min", "max"):
        assert got["f64"] == exp.f64, f"{ctx}: {got['f64']!r} != {exp.f64!r}"
        return {}
    # float SUM / AVG
    assert got["prec_used"] == {"neumaier": 0, "f32": 1, "f64_combine": 2}[prec], ctx
    exact_sum = oracle.aggregate(x, oracle.SUM, threads).f64
    abs_sum = oracle.aggregate(x, oracle.ABS_SUM, threads).f64
    bound = float_sum_bound(prec, n, abs_sum)
    if op == "sum":
        err = abs(got["f64"] - exact_sum)
        rep = oracle.error_report(got["f64"], exact_sum, abs_sum)
    else:
        err = abs(got["f64"] - exact_sum / n) * n
        rep = oracle.error_report(got["f64"] * n, exact_sum, abs_sum)
        bound += 4 * U64 * abs(exact_sum)
    assert err <= bound, f"{ctx}: |err| {err!r} > bound {bound!r} (S*={exact_sum!r}, A={abs_sum!r})"
    if prec == "neumaier" and exact_sum != 0 and rep["kappa"] < 1e6:
        assert rep["rel"] <= REL_GATE_COMPENSATED, f"{ctx}: rel {rep['rel']} > 1e-6"
    rep["bound_abs"] = bound
    return rep


def same_bits(a: dict, b: dict) -> bool:
    def key(d):
        f = d["f64"]
        return (d["i64"], struct_bits(f), d["count"], d["is_null"], d["prec_used"])
    return key(a) == key(b)


def struct_bits(f: float) -> int:
    return int(np.array([f], dtype=np.float64).view(np.int64)[0])
