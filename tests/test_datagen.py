"""The seeded input generators: determinism, ranges and distribution shapes."""
import math

import numpy as np
import pytest

import datagen


def test_splitmix64_reference_values():
    # The finaliser against a plain-Python evaluation of the published mix.
    for seed in (0, 1, 12345, 2**63 + 7):
        key = datagen.splitmix64_mix(seed ^ datagen.splitmix64_mix(
            (0 * 0x9E3779B97F4A7C15 + 0x5851F42D4C957F2D) & (2**64 - 1)))
        for ctr in (0, 1, 2, 1000, 2**40):
            want = datagen.splitmix64_mix(key + (ctr + 1) * 0x9E3779B97F4A7C15)
            assert datagen.raw(seed, ctr) == want
    # SplitMix64's known first output for state 0 + gamma (Vigna's reference code).
    assert datagen.splitmix64_mix(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("dtype", ["i32", "i64", "f32"])
@pytest.mark.parametrize("dist", ["uniform", "zipf", "sorted"])
def test_deterministic_and_thread_invariant(dtype, dist):
    a = datagen.column(300_001, dtype, dist, seed=9, threads=1)
    b = datagen.column(300_001, dtype, dist, seed=9, threads=7)
    c = datagen.column(300_001, dtype, dist, seed=10, threads=4)
    assert a.tobytes() == b.tobytes()
    assert a.tobytes() != c.tobytes()
    # a prefix of a longer column is the shorter column (counter based)
    if dist != "sorted":
        d = datagen.column(1000, dtype, dist, seed=9)
        assert d.tobytes() == a[:1000].tobytes()


def test_uniform_ranges():
    x = datagen.column(1_000_000, "i32", "uniform", seed=2)
    assert x.min() >= -2**20 and x.max() < 2**20 and x.min() < -2**20 + 100 and x.max() > 2**20 - 100
    y = datagen.column(1_000_000, "i64", "uniform", seed=3)
    assert y.min() >= -2**32 and y.max() < 2**32 and y.max() > 2**31
    z = datagen.column(1_000_000, "f32", "uniform", seed=4)
    assert z.min() >= -2**20 and z.max() < 2**20
    assert np.all(z.astype(np.float64) * 8 == np.round(z.astype(np.float64) * 8))  # 1/8 grid
    w = datagen.column(1_000_000, "i32", "uniform", seed=5, lo=1, hi=2_000_001)
    assert w.min() >= 1 and w.max() <= 2_000_000
    # mean of a uniform on [-2^20, 2^20): about -0.5 +- 4 sigma
    sigma = 2**21 / math.sqrt(12) / math.sqrt(x.size)
    assert abs(x.astype(np.float64).mean() + 0.5) < 5 * sigma


@pytest.mark.parametrize("dtype", ["i32", "i64", "f32"])
def test_sorted_is_sorted_permutation_of_uniform(dtype):
    u = datagen.column(500_003, dtype, "uniform", seed=6)
    s = datagen.column(500_003, dtype, "sorted", seed=6, threads=5)
    assert np.all(s[1:] >= s[:-1])
    assert np.array_equal(np.sort(u), s)


def test_sorted_custom_range():
    u = datagen.column(200_000, "i64", "uniform", seed=8, lo=1, hi=10**6 + 1)
    s = datagen.column(200_000, "i64", "sorted", seed=8, lo=1, hi=10**6 + 1)
    assert np.array_equal(np.sort(u), s)


def test_zipf_shape():
    x = datagen.column(2_000_000, "i32", "zipf", seed=7)
    assert x.min() >= 1 and x.max() <= 2**20
    h = sum(k ** -1.1 for k in range(1, 2**20 + 1))
    for k in (1, 2, 3, 10):
        p = k ** -1.1 / h
        f = np.count_nonzero(x == k) / x.size
        assert abs(f - p) < 6 * math.sqrt(p * (1 - p) / x.size)
    f = datagen.column(1000, "f32", "zipf", seed=7)
    assert np.array_equal(f, x[:1000].astype(np.float32))


def test_normal_outliers_shape():
    x = datagen.column(2_000_000, "f32", "normal_outliers", seed=11)
    big = np.abs(x) == np.float32(1e6)
    frac = big.mean()
    assert abs(frac - 0.01) < 6 * math.sqrt(0.01 * 0.99 / x.size)
    assert abs((x[big] > 0).mean() - 0.5) < 0.02
    body = x[~big].astype(np.float64)
    assert abs(body.mean()) < 0.01 and abs(body.std() - 1.0) < 0.01
    assert np.abs(body).max() < 7


def test_invalid_arguments():
    with pytest.raises(ValueError):
        datagen.column(10, "i32", "normal_outliers", seed=1)
    with pytest.raises(ValueError):
        datagen.column(10, "f32", "uniform", seed=1, lo=1, hi=5)
    with pytest.raises(ValueError):
        datagen.column(10, "i32", "uniform", seed=1, lo=5, hi=5 - 10)
