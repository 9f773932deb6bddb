"""Shared checks of GPU results against the CPU oracle.

Integer SUM / MIN / MAX / COUNT / AVG and float MIN / MAX must match the oracle
bit for bit.  Float SUM / AVG must lie within the a-priori error bound of the
precision mode for the canonical reduction shape, derived below; the
compensated mode must in addition be within 1e-6 relative of the exact sum.

Notation: u = 2^-24 (float32 unit roundoff), v = 2^-53 (double), A = sum |x_i|,
gamma_d(w) = d w / (1 - d w).  The canonical shape has segments of S bytes; a
lane accumulator (one vector component of one lane) folds m <= S / 1024 items;
each segment's accumulators merge over 8 tree levels (2 component levels, 6
butterfly levels); nseg segment partials merge over k - 1 sequential additions
(k = ceil(nseg / 256) per lane of the final combine; the first addition to the
zero identity is exact) plus 8 tree levels (6 butterfly, 2 across the four
waves).

  plain f32     every addition is one float32 rounding and no item passes
                through more than m + k + 16 of them, so (Higham, Accuracy and
                Stability of Numerical Algorithms, 2nd ed., Section 4.2; the
                bound for any summation tree of depth d is gamma_d times A):
                |err| <= gamma_{m+k+18}(u) A
  f64 combine   float32 up to the segment total (depth <= m + 8), exact
                widening, then the double combine (depth k + 7) over partials
                whose magnitudes sum to at most (1 + gamma_{m+8}(u)) A:
                |err| <= gamma_{m+8}(u) A + gamma_{k+8}(v) (1 + gamma_{m+8}(u)) A
  Neumaier      each accumulator (s, c) satisfies s + c = (exact running sum) +
                (the rounding errors of c's own additions): Neumaier's step
                and the two-sums are exact.  Every R = 8 rounds the pair is
                renormalised by an exact two-sum, after which |c| <= u |s|
                <= u Ab (Ab ~ A, the accumulator's sum of |x|, to 1 + 1e-6 for
                any shape here).  Within a block, the j-th correction addition
                adds at most u (j + 1) u Ab, so a block of b <= R items adds at
                most b (b + 3) / 2 u^2 Ab, and at most ceil(m / R) blocks make
                the lane error <= ceil(m / R) R (R + 3) / 2 u^2 Ab.  A pair merge
                (two-sum of the s parts, corrections added, renormalised) adds
                at most 3 u^2 (A1 + A2), so the 8 merge levels add 24 u^2 A;
                forming s + c in double adds v |S_seg|; the double combine adds
                gamma_{k+7}(v) times the partials' magnitudes:
                |err| <= 1.01 [(ceil(m/R) R (R+3)/2 + 24) u^2 + (k + 8) v] A
                The factor 1.01 covers every (1 + O(u)) factor (each below
                1 + 1e-6 for m <= 2^14).  Without the renormalisation the
                correction term of the published bound for cascaded summation
                (Ogita, Rump and Oishi, SIAM J. Sci. Comput. 26(6), 2005,
                Prop. 4.5: |err| <= u |S| + gamma_{n-1}(u)^2 A) is quadratic in
                m: at m = 512, about 2.6e5 u^2 A against 2840 u^2 A here.
The tests check these bounds as stated (they are worst-case, not estimates).
"""
from __future__ import annotations

import math

import numpy as np

import oracle

U32 = 2.0 ** -24
U64 = 2.0 ** -53
REL_GATE_COMPENSATED = 1e-6
NEU_RENORM_ROUNDS = 8

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


def gamma(d: int, w: float) -> float:
    return d * w / (1.0 - d * w)


def float_sum_bound_coeff(prec: str, n: int) -> float:
    """The a-priori bound of |computed - exact| as a multiple of sum |x| for
    a float32 column of n items in precision mode `prec`."""
    seg = seg_bytes_for(4, n)
    m = seg // 1024
    nseg = -(-(n * 4) // seg) if n else 0
    k = -(-nseg // 256) if nseg else 0
    if prec == "f32":
        return gamma(m + k + 18, U32)
    if prec == "f64_combine":
        g = gamma(m + 8, U32)
        return g + gamma(k + 8, U64) * (1.0 + g)
    r = NEU_RENORM_ROUNDS
    lane = -(-m // r) * r * (r + 3) / 2
    return 1.01 * ((lane + 24) * U32 * U32 + (k + 8) * U64)


def float_sum_bound(prec: str, n: int, abs_sum: float) -> float:
    return float_sum_bound_coeff(prec, n) * abs_sum


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
