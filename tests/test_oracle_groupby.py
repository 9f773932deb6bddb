"""Pins of the group-by oracle: brute force with Python dicts, integers and
exact rationals; invariants against the whole-column oracle."""
import math
from collections import defaultdict
from fractions import Fraction

import numpy as np
import pytest

import oracle

M64 = 1 << 64


def wrap64(v):
    v %= M64
    return v - M64 if v >= 1 << 63 else v


def brute(keys, vals, op):
    g = defaultdict(list)
    for k, v in zip(keys.tolist(), vals.tolist()):
        g[k].append(v)
    out = []
    for k in sorted(g):
        xs = g[k]
        c = len(xs)
        if vals.dtype == np.float32:
            if op == "count":
                out.append((k, c, float(c), c))
                continue
            exact = sum((Fraction(x) for x in xs), Fraction(0))
            s = exact.numerator / exact.denominator
            f = {"sum": s, "avg": s / c, "min": min(xs), "max": max(xs)}[op]
            out.append((k, 0, f, c))
        else:
            if op == "count":
                out.append((k, c, float(c), c))
                continue
            s = wrap64(sum(xs))
            iv = {"sum": s, "avg": s, "min": min(xs), "max": max(xs)}[op]
            fv = float(s) / c if op == "avg" else float(iv)
            out.append((k, iv, fv, c))
    return out


@pytest.mark.parametrize("kdt", [np.int32, np.int64])
@pytest.mark.parametrize("vdt", [np.int32, np.int64, np.float32])
@pytest.mark.parametrize("op", ["sum", "min", "max", "count", "avg"])
def test_groupby_brute_force(kdt, vdt, op):
    r = np.random.default_rng(hash((str(kdt), str(vdt), op)) % 2**32)
    for n, card in [(0, 1), (1, 1), (7, 3), (1000, 10), (5000, 4000)]:
        keys = r.integers(-card, card, size=n).astype(kdt)
        if vdt == np.float32:
            vals = (r.standard_normal(n) * np.exp2(r.integers(-30, 31, size=n))).astype(np.float32)
        else:
            info = np.iinfo(vdt)
            vals = r.integers(info.min, info.max, size=n, dtype=np.int64).astype(vdt)
        assert oracle.groupby(keys, vals, op) == brute(keys, vals, op)


def test_groupby_invariants():
    r = np.random.default_rng(5)
    n = 200_000
    keys = r.integers(0, 5000, size=n).astype(np.int64)
    vals = r.integers(-2**40, 2**40, size=n).astype(np.int64)
    g = oracle.groupby(keys, vals, "sum")
    assert len(g) == len(np.unique(keys))
    assert sum(c for _, _, _, c in g) == n
    assert wrap64(sum(s for _, s, _, _ in g)) == oracle.value(vals, "sum")
    assert min(m for _, m, _, _ in oracle.groupby(keys, vals, "min")) == oracle.value(vals, "min")
    assert max(m for _, m, _, _ in oracle.groupby(keys, vals, "max")) == oracle.value(vals, "max")
    assert [k for k, *_ in g] == sorted(set(keys.tolist()))


def test_single_group_equals_whole_column():
    r = np.random.default_rng(6)
    x = (r.standard_normal(100_003) * 1e3).astype(np.float32)
    k = np.full(x.size, 42, np.int32)
    (key, _, s, c), = oracle.groupby(k, x, "sum")
    assert key == 42 and c == x.size and s == oracle.value(x, "sum")
    xi = r.integers(-2**31, 2**31, size=77_777, dtype=np.int64).astype(np.int32)
    (_, si, fa, _), = oracle.groupby(np.zeros(xi.size, np.int64), xi, "avg")
    assert fa == oracle.value(xi, "avg") and si == oracle.value(xi, "sum")


def test_extreme_keys():
    keys = np.array([-2**63, 2**63 - 1, -2**63, 0], np.int64)
    vals = np.array([1, 2, 3, 4], np.int32)
    assert oracle.groupby(keys, vals, "sum") == [(-2**63, 4, 4.0, 2), (0, 4, 4.0, 1), (2**63 - 1, 2, 2.0, 1)]
