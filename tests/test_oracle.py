"""Pins of the CPU oracle against things other than itself.

The paper prints no per-value results for aggregation (its only numbers are
throughputs and energies of whole runs), so every pin comes from mathematics:
brute force with Python integers and exact rationals, the correctly rounded
``math.fsum``, closed forms (sum of 0..n-1, constants, cancellation patterns),
special cases of IEEE rounding, and invariants (permutation, thread count,
additivity, min <= avg <= max).  Each pin is chosen to catch a plausible
mistake: a dropped or duplicated item, a wrong sign, a lost carry, a
truncating instead of rounding conversion, a narrowed accumulator.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import datagen
import oracle
from oracle import AVG, COUNT, F32, I32, I64, MAX, MIN, SUM

SIZES = [0, 1, 2, 3, 4, 5, 63, 64, 65, 1000, 1_000_003]
M64 = 1 << 64


def wrap64(v: int) -> int:
    v %= M64
    return v - M64 if v >= (1 << 63) else v


def rng(seed):
    return np.random.default_rng(seed)


def correctly_rounded(fr: Fraction) -> float:
    # int / int true division in CPython is correctly rounded (ties to even).
    return fr.numerator / fr.denominator


# --------------------------------------------------------------- integers
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dt,lo,hi", [(np.int32, -2**31, 2**31), (np.int64, -2**62, 2**62)])
def test_int_sum_min_max_brute_force(n, dt, lo, hi):
    x = rng(n + 7).integers(lo, hi, size=n, dtype=dt)
    py = [int(v) for v in x]
    r = oracle.aggregate(x, "sum")
    assert r.i64 == wrap64(sum(py)) and r.count == n and not r.is_null
    if n:
        assert oracle.value(x, "min") == min(py)
        assert oracle.value(x, "max") == max(py)
        assert oracle.value(x, "avg") == float(wrap64(sum(py))) / float(n)
    else:
        assert oracle.value(x, "min") is None and oracle.value(x, "max") is None
        assert oracle.value(x, "avg") is None
    assert oracle.value(x, "count") == n


def test_int64_sum_wraps_mod_2_64():
    x = np.array([2**63 - 1, 1, 2**63 - 1, 5], dtype=np.int64)
    assert oracle.value(x, "sum") == wrap64(2**63 - 1 + 1 + 2**63 - 1 + 5)
    y = np.full(4, -2**63, dtype=np.int64)
    assert oracle.value(y, "sum") == 0


@pytest.mark.parametrize("n", [1, 2, 1000, 1_000_003])
def test_int_closed_forms(n):
    a = np.arange(n, dtype=np.int32)
    assert oracle.value(a, "sum") == n * (n - 1) // 2
    assert oracle.value(a, "min") == 0 and oracle.value(a, "max") == n - 1
    assert oracle.value(a, "avg") == (n - 1) / 2
    # a column of INT32_MIN only sums correctly if the accumulator is 64 bits
    m = np.full(n, -2**31, dtype=np.int32)
    assert oracle.value(m, "sum") == n * -2**31
    c = np.full(n, 12345, dtype=np.int64)
    assert oracle.value(c, "sum") == 12345 * n and oracle.value(c, "avg") == 12345.0
    alt = np.where(np.arange(n) % 2 == 0, 1, -1).astype(np.int32)
    assert oracle.value(alt, "sum") == (n % 2)


def test_planted_extremes_found_anywhere():
    r = rng(3)
    for trial in range(20):
        n = int(r.integers(1, 200_000))
        x = r.integers(-1000, 1000, size=n, dtype=np.int64)
        i, j = int(r.integers(0, n)), int(r.integers(0, n))
        x[i] = -2**63
        x[j] = 2**63 - 1 if j != i else x[j]
        assert oracle.value(x, "min") == -2**63
        if j != i:
            assert oracle.value(x, "max") == 2**63 - 1


def test_int_invariants_permutation_threads_additivity():
    x = rng(11).integers(-2**20, 2**20, size=1_000_003, dtype=np.int32)
    ref = oracle.aggregate(x, SUM, threads=1).i64
    for t in (2, 3, 8, 16):
        assert oracle.aggregate(x, SUM, threads=t).i64 == ref
    assert oracle.value(rng(12).permutation(x), "sum") == ref
    k = 400_001
    assert oracle.value(x[:k], "sum") + oracle.value(x[k:], "sum") == ref
    mn, mx, av = oracle.value(x, "min"), oracle.value(x, "max"), oracle.value(x, "avg")
    assert mn <= av <= mx


# --------------------------------------------------------------- float32
def f32_exact(x: np.ndarray) -> Fraction:
    return sum((Fraction(float(v)) for v in x), Fraction(0))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 64, 65, 300])
@pytest.mark.parametrize("scale", ["unit", "wide", "subnormal"])
def test_f32_sum_is_exact_sum_rounded_once(n, scale):
    r = rng(n * 31 + len(scale))
    if scale == "unit":
        x = r.standard_normal(n).astype(np.float32)
    elif scale == "wide":  # magnitudes 2^-60 .. 2^60, both signs: heavy cancellation
        x = (r.standard_normal(n) * np.exp2(r.integers(-60, 61, size=n))).astype(np.float32)
    else:  # subnormal and tiny normals
        x = (r.integers(-2**23, 2**23, size=n).astype(np.float64) * 2.0**-149).astype(np.float32)
    got = oracle.value(x, "sum")
    assert got == correctly_rounded(f32_exact(x))
    assert oracle.value(x, "abs_sum") == correctly_rounded(f32_exact(np.abs(x)))


@pytest.mark.parametrize("n", [1000, 100_003, 1_000_003])
def test_f32_sum_matches_fsum(n):
    r = rng(n)
    x = np.concatenate([r.standard_normal(n - n // 100),
                        np.where(r.random(n // 100) < 0.5, -1e6, 1e6)]).astype(np.float32)
    r.shuffle(x)
    assert oracle.value(x, "sum") == math.fsum(float(v) for v in x)
    assert oracle.value(x, "avg") == math.fsum(float(v) for v in x) / n


def test_f32_closed_forms():
    ones = np.ones(2**24, dtype=np.float32)
    assert oracle.value(ones, "sum") == 2.0**24
    m = 100_000
    canc = np.tile(np.array([1e8, 1.0, -1e8], dtype=np.float32), m)
    assert oracle.value(canc, "sum") == float(m)   # plain float32 summation gives 0
    n = 2**20
    ar = np.arange(n, dtype=np.float32)
    assert oracle.value(ar, "sum") == n * (n - 1) / 2
    pm = np.tile(np.array([1e6, -1e6], dtype=np.float32), 50_000)
    rng(5).shuffle(pm)
    assert oracle.value(pm, "sum") == 0.0
    big = np.full(3, np.finfo(np.float32).max, dtype=np.float32)
    assert oracle.value(big, "sum") == 3.0 * float(np.finfo(np.float32).max)
    assert oracle.value(-big, "sum") == -3.0 * float(np.finfo(np.float32).max)


def test_f32_rounding_ties_and_sticky_bits():
    two53 = np.float32(2.0**53)
    # exact 2^53 + 1 is a tie between 2^53 and 2^53 + 2: even wins
    assert oracle.value(np.array([two53, 1.0], np.float32), "sum") == 2.0**53
    # 2^53 + 3 is a tie between +2 and +4: even mantissa is +4
    assert oracle.value(np.array([two53, 1.0, 2.0], np.float32), "sum") == 2.0**53 + 4
    # a bit below the tie point (the sticky bit) forces rounding up
    assert oracle.value(np.array([two53, 1.0, 2.0**-20], np.float32), "sum") == 2.0**53 + 2
    # and negative sums round symmetrically
    assert oracle.value(np.array([-two53, -1.0, -2.0**-20], np.float32), "sum") == -(2.0**53 + 2)
    assert oracle.value(np.array([-two53, -1.0], np.float32), "sum") == -(2.0**53)


def test_f32_nonfinite_and_empty():
    assert math.isnan(oracle.value(np.array([1, np.nan], np.float32), "sum"))
    assert math.isnan(oracle.value(np.array([np.inf, -np.inf], np.float32), "sum"))
    assert oracle.value(np.array([np.inf, 1], np.float32), "sum") == math.inf
    assert oracle.value(np.array([3, np.nan, -2], np.float32), "min") == -2.0
    assert oracle.value(np.array([3, np.nan, -2], np.float32), "max") == 3.0
    assert math.isnan(oracle.value(np.array([np.nan], np.float32), "min"))
    e = np.zeros(0, np.float32)
    assert oracle.value(e, "sum") == 0.0 and oracle.value(e, "count") == 0
    assert oracle.value(e, "min") is None and oracle.value(e, "avg") is None


def test_f32_min_max_brute_force():
    r = rng(21)
    for n in (1, 2, 65, 5000, 1_000_003):
        x = r.standard_normal(n).astype(np.float32) * 1e3
        assert oracle.value(x, "min") == float(min(x.tolist()))
        assert oracle.value(x, "max") == float(max(x.tolist()))


def test_f32_invariants_threads_and_permutation():
    r = rng(22)
    n = 3_000_017
    x = (r.standard_normal(n) * np.exp2(r.integers(-30, 31, size=n))).astype(np.float32)
    ref = oracle.aggregate(x, SUM, threads=1).f64
    for t in (2, 7, 16):
        assert oracle.aggregate(x, SUM, threads=t).f64 == ref
    assert oracle.value(r.permutation(x), "sum") == ref
    assert ref == math.fsum(x.astype(np.float64).tolist())


def test_error_report():
    rep = oracle.error_report(1.5, 1.0, 4.0)
    assert rep["rel"] == 0.5 and rep["abs_norm"] == 0.125 and rep["kappa"] == 4.0
    assert oracle.error_report(0.0, 0.0, 1.0)["rel"] is None


def test_superaccumulator_digit_headroom():
    # Every addition of a float near FLT_MAX lands in the top digits; 2^25 of
    # them with alternating signs must cancel exactly down to the last item.
    n = 2**25
    fmax = np.finfo(np.float32).max
    x = np.full(n, fmax, dtype=np.float32)
    x[1::2] *= -1
    x[-1] = np.float32(1.0)  # n even: all pairs cancel except one +FLT_MAX
    exp = correctly_rounded(Fraction(float(fmax)) + 1)
    assert oracle.value(x, "sum") == exp
    assert oracle.value(x[:-1], "sum") == float(fmax)


# ---- block tables and sub-range aggregation (for checking many ranges of one large column)
@pytest.mark.parametrize("dtype", ["i32", "i64"])
def test_block_table_is_the_per_block_definition(dtype):
    x = datagen.column(100_003, dtype, "uniform", seed=31)
    x[4321] = np.iinfo(x.dtype).min
    x[99_999] = np.iinfo(x.dtype).max
    for block in (1, 7, 1000, 65536, 200_000):
        for op, f in (("sum", lambda v: int(np.sum(v.astype(np.int64)))), ("min", lambda v: int(v.min())),
                      ("max", lambda v: int(v.max()))):
            t = oracle.block_table(x, op, block, threads=3)
            want = [f(x[j:j + block]) for j in range(0, x.size, block)]
            assert t.tolist() == want, (dtype, block, op)


@pytest.mark.parametrize("dtype", ["i32", "i64"])
def test_range_oracle_equals_whole_slice_oracle(dtype):
    n = 1_000_003
    x = datagen.column(n, dtype, "uniform", seed=32)
    ro = oracle.RangeOracle(x.ctypes.data, n, oracle.DTYPES[dtype], block=4096, threads=4)
    rng = np.random.default_rng(5)
    ranges = [(0, 0), (0, n), (5, 1), (4096, 4096), (4095, 2), (4096 * 3 - 1, 4096 * 5 + 2), (n - 17, 17)]
    for _ in range(40):
        off = int(rng.integers(0, n))
        ranges.append((off, int(rng.integers(0, n - off + 1))))
    for off, m in ranges:
        for op in ("sum", "min", "max", "count", "avg"):
            got = ro.aggregate(off, m, op)
            want = oracle.aggregate(x[off:off + m], op)
            assert (got.i64, got.count, got.is_null) == (want.i64, want.count, want.is_null), (off, m, op)
            assert got.f64 == want.f64 or (np.isnan(got.f64) and np.isnan(want.f64)), (off, m, op)


def test_range_oracle_wraps_like_the_oracle():
    x = np.full(300_000, np.iinfo(np.int64).max, dtype=np.int64)
    ro = oracle.RangeOracle(x.ctypes.data, x.size, oracle.I64, block=1000)
    for off, m in ((0, 300_000), (17, 123_456)):
        assert ro.aggregate(off, m, "sum").i64 == oracle.aggregate(x[off:off + m], "sum").i64


def test_read_ceiling_reads_every_word():
    b = np.random.default_rng(3).integers(0, 2 ** 63, size=100_001, dtype=np.int64).view(np.uint64)
    for threads in (1, 3, 8):
        assert oracle.read_ceiling(b.ctypes.data, b.nbytes, threads) == int(np.bitwise_xor.reduce(b))
