"""The float32 SUM error bounds of `aggcheck.py`, exercised on the CPU.

* The compensated lane fold (Neumaier's update, exact two-sum renormalisation
  every 8 rounds), modelled step by step in numpy float32, stays within the
  linear per-lane bound ceil(m/8) * 44 * u^2 * sum|x| on inputs built to make
  the correction's own roundings add up; without the renormalisation the same
  inputs exceed that bound (the quadratic term of the cascaded-summation bound
  of Ogita, Rump and Oishi 2005, Prop. 4.5, is real).
* The whole canonical shape (lanes, merges, double combine) stays within the
  stated bound of each precision mode against the exact sum of the oracle.
* At the benchmark's full sizes (2^30 float32 items), the a-priori relative
  bound of the compensated mode is <= 1e-6 for every float32 column the
  benchmark and the full-size GPU tests use: the uniform columns (seeds 4, 8
  and 10; the sorted column of seed 10 is a permutation of the uniform one,
  `test_datagen.py`, so its exact sum and sum|x| are the same), Zipf (seed 9)
  and N(0,1) with 1% of +-1e6 (seed 11).
"""
import math

import numpy as np
import pytest

import datagen
import oracle
import shape_model as sm
from aggcheck import NEU_RENORM_ROUNDS, U32, float_sum_bound, float_sum_bound_coeff

M = 512        # items per lane accumulator at 2^30 float32 items (512 KiB segments)
LANES = 1024


def lane_bound_coeff(m, r=NEU_RENORM_ROUNDS):
    return -(-m // r) * r * (r + 3) / 2 * U32 * U32


def adversarial_rounds(kind, seed):
    """Rounds (M, LANES) of float32 items for independent accumulators."""
    rng = np.random.default_rng(seed)
    x = np.empty((M, LANES), np.float32)
    big = (2.0 ** 24 * (1 + rng.integers(0, 2 ** 23, LANES) * 2.0 ** -23)).astype(np.float32)
    x[0] = big * np.where(rng.integers(0, 2, LANES) == 1, 1, -1).astype(np.float32)
    if kind == "below_half_ulp":
        # every later item is below half an ulp of the running sum: s never
        # moves, each item is an exact rounding error, and the correction sums
        # them in float32
        x[1:] = rng.uniform(0.5, 0.999, (M - 1, LANES)).astype(np.float32)
    elif kind == "mixed_scales":
        x[1:] = (rng.uniform(1, 2, (M - 1, LANES)) * 2.0 ** rng.integers(-12, 0, (M - 1, LANES))).astype(np.float32)
    elif kind == "cancelling_outliers":
        x[1:] = rng.standard_normal((M - 1, LANES)).astype(np.float32)
        hit = rng.random((M - 1, LANES)) < 0.05
        x[1:][hit] = (np.where(rng.random(hit.sum()) < 0.5, 1, -1) * 1e6).astype(np.float32)
    return x


def worst_ratio(x, renorm):
    """max over accumulators of |s + c - exact| / (u^2 sum|x|)."""
    s, c = sm.lane_fold_neumaier(x, renorm=renorm)
    worst = 0.0
    for l in range(x.shape[1]):
        col = x[:, l].astype(np.float64)
        err = abs(math.fsum([float(s[l]), float(c[l])] + [-v for v in col]))
        worst = max(worst, err / (U32 * U32 * math.fsum(np.abs(col))))
    return worst


@pytest.mark.parametrize("kind", ["below_half_ulp", "mixed_scales", "cancelling_outliers"])
def test_renormalised_lane_fold_within_linear_bound(kind):
    x = adversarial_rounds(kind, seed=5)
    ratio = worst_ratio(x, NEU_RENORM_ROUNDS)
    assert ratio * U32 * U32 <= lane_bound_coeff(M), (kind, ratio)


def test_unrenormalised_correction_exceeds_linear_bound():
    """The variant without renormalisation: the correction's roundings grow
    past the linear bound (so the renormalisation is what makes it hold)."""
    x = adversarial_rounds("below_half_ulp", seed=5)
    ratio = worst_ratio(x, 0)
    assert ratio * U32 * U32 > 2 * lane_bound_coeff(M), ratio


@pytest.mark.parametrize("prec", ["neumaier", "f64_combine", "f32"])
@pytest.mark.parametrize("dist,seed", [("normal_outliers", 11), ("uniform", 3), ("zipf", 4)])
@pytest.mark.parametrize("n", [1, 7, 1000, (1 << 16) + 3, (3 << 20) + 7])
def test_model_within_stated_bound(prec, dist, seed, n):
    x = datagen.column(n, "f32", dist, seed=seed)
    exact = oracle.aggregate(x, "sum").f64
    a = oracle.aggregate(x, "abs_sum").f64
    got = sm.model_sum(x, prec)
    # the exact sum is itself rounded to double once: allow its half ulp
    assert abs(got - exact) <= float_sum_bound(prec, n, a) + 2.0 ** -53 * abs(exact), (got, exact)


def test_model_compensation_cancels_exactly():
    """[1e8, 1, -1e8] * k: plain float32 loses every 1, the compensated mode keeps them."""
    k = 5000
    x = np.tile(np.array([1e8, 1.0, -1e8], np.float32), k)
    assert sm.model_sum(x, "neumaier") == float(k)
    assert sm.model_sum(x, "f32") != float(k)


@pytest.mark.slow
@pytest.mark.parametrize("dist,seed", [("uniform", 4), ("uniform", 8), ("uniform", 10), ("zipf", 9),
                                       ("normal_outliers", 11)])
def test_full_size_columns_have_apriori_relative_bound_below_1e6(dist, seed):
    n = 1 << 30
    x = datagen.column(n, "f32", dist, seed=seed)
    exact = oracle.aggregate(x, "sum").f64
    a = oracle.aggregate(x, "abs_sum").f64
    del x
    rel = float_sum_bound_coeff("neumaier", n) * a / abs(exact)
    assert rel <= 1e-6, f"{dist} seed {seed}: a-priori relative bound {rel:.3e} (kappa {a / abs(exact):.3e})"


@pytest.mark.slow
def test_stored_precision_refs_match_the_oracle():
    """The benchmark's stored exact sums (tests/golden/precision_refs.json)
    are what the oracle computes for those columns."""
    import json
    import os
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    import make_precision_refs as mk
    stored = json.load(open(os.path.join(here, "golden", "precision_refs.json")))["columns"]
    assert set(stored) == {name for name, _, _ in mk.COLUMNS}
    for name, dist, seed in mk.COLUMNS:
        assert stored[name] == mk.compute(dist, seed), name


@pytest.mark.parametrize("n", [0, 1, 1000, (1 << 20) + 3, 1 << 26, 1 << 30, (1 << 32) + 5])
@pytest.mark.parametrize("prec", ["neumaier", "f64_combine", "f32"])
def test_library_states_the_same_bound(prec, n):
    """The bound the library documents (and the benchmark reports) is the one
    the tests hold the GPU to."""
    import paper_2606_10030_amd as agg
    if n == 0:
        return
    assert agg.float_sum_bound_coeff(prec, n) == pytest.approx(float_sum_bound_coeff(prec, n), rel=1e-12)
