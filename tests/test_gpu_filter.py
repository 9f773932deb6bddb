"""GPU: fused filter + aggregate (agg_run_filtered).

Reference: the oracle on the selected items x[mask], with the mask taken
from the predicate's definition (numpy comparisons of the filter column in
int64 / float64).  Always-true predicates must give agg_run's bits; empty
selections give null MIN / MAX / AVG and zero SUM / COUNT."""
import numpy as np
import pytest

import datagen
import oracle
from aggcheck import check, same_bits

pytestmark = pytest.mark.gpu

DTS = ["i32", "i64", "f32"]
OPS = ["sum", "min", "max", "count", "avg"]


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    return agg


def mask_of(y, lo, hi, lo_inc, hi_inc):
    yy = y.astype(np.float64) if y.dtype == np.float32 else y.astype(np.int64)
    m = np.ones(y.size, bool)
    if lo is not None:
        m &= (yy >= lo) if lo_inc else (yy > lo)
    if hi is not None:
        m &= (yy <= hi) if hi_inc else (yy < hi)
    return m


def check_selected(x, m, dtype, op, prec, got, ctx):
    sel = np.ascontiguousarray(x[m])
    r = dict(got)
    assert r["count"] == sel.size, f"{ctx}: selected {r['count']} != {sel.size}"
    check(sel, dtype, op, prec, r, ctx=ctx)


@pytest.mark.parametrize("vdt", DTS)
@pytest.mark.parametrize("fdt", DTS)
def test_filtered_matches_oracle(agg, vdt, fdt):
    import torch
    n = 3_000_017
    r = np.random.default_rng(hash((vdt, fdt)) % 2**32)
    if vdt == "f32":
        x = (r.standard_normal(n) * np.exp2(r.integers(-20, 21, size=n))).astype(np.float32)
    else:
        x = datagen.column(n, vdt, "uniform", seed=3)
    y = datagen.column(n, fdt, "uniform", seed=4)
    dx, dy = torch.from_numpy(x).to("cuda"), torch.from_numpy(y).to("cuda")
    preds = [(-1000, 1000, True, False), (0, None, True, True), (None, -5, True, False),
             (12345, 12345, True, True), (2**21, None, True, True)]      # the last selects nothing
    precs = ["neumaier", "f32", "f64_combine"] if vdt == "f32" else ["neumaier"]
    for lo, hi, li, hi_inc in preds:
        m = mask_of(y, lo, hi, li, hi_inc)
        filt = agg.make_filter(dy, lo, hi, li, hi_inc)
        for op in OPS:
            for prec in precs if op in ("sum", "avg") else ["neumaier"]:
                got = agg.Plan(vdt, op, max_n=n, prec=prec).run_filtered(dx, filt)
                check_selected(x, m, vdt, op, prec, got, f"{vdt}<-{fdt} [{lo},{hi}] {op} {prec}")


@pytest.mark.parametrize("vdt", DTS)
def test_always_true_equals_agg_run(agg, vdt):
    import torch
    for n in (0, 1, 63, 1025, 65_539, 2_000_003):
        if vdt == "f32":
            r = np.random.default_rng(n)
            x = (r.standard_normal(n) * np.exp2(r.integers(-20, 21, size=n))).astype(np.float32)
        else:
            x = datagen.column(n, vdt, "uniform", seed=n)
        y = datagen.column(n, "i32", "uniform", seed=n + 1)
        dx, dy = torch.from_numpy(x).to("cuda"), torch.from_numpy(y).to("cuda")
        for op in OPS:
            for prec in ("neumaier", "f32", "f64_combine") if vdt == "f32" and op in ("sum", "avg") else ("neumaier",):
                p = agg.Plan(vdt, op, max_n=max(n, 1), prec=prec)
                a = p.run(dx, n=n)
                b = p.run_filtered(dx, agg.make_filter(dy), n=n)
                assert same_bits(a, b), f"{vdt} {op} {prec} n={n}: always-true filter differs from agg_run"


def test_unaligned_columns(agg):
    import torch
    n = 1_000_003
    x = datagen.column(n + 3, "i64", "uniform", seed=8)
    y = datagen.column(n + 3, "f32", "uniform", seed=9)
    dx, dy = torch.from_numpy(x).to("cuda"), torch.from_numpy(y).to("cuda")
    for ox, oy in ((1, 0), (0, 1), (1, 3)):
        vx, vy = dx[ox:ox + n], dy[oy:oy + n]
        m = mask_of(y[oy:oy + n], -1e5, 1e5, True, True)
        for op in ("sum", "min", "max", "count"):
            got = agg.Plan("i64", op, max_n=n).run_filtered(vx, agg.make_filter(vy, -1e5, 1e5))
            check_selected(x[ox:ox + n], m, "i64", op, "neumaier", got, f"unaligned ({ox},{oy}) {op}")


def test_nan_filter_items_are_never_selected(agg):
    import torch
    x = np.arange(10_000, dtype=np.int32)
    y = np.zeros(10_000, np.float32)
    y[::3] = np.nan
    got = agg.Plan("i32", "count", max_n=x.size).run_filtered(
        torch.from_numpy(x).to("cuda"), agg.make_filter(torch.from_numpy(y).to("cuda")))
    assert got["i64"] == int(np.count_nonzero(~np.isnan(y)))


def test_filter_errors(agg):
    import torch
    x = torch.arange(1000, dtype=torch.int32, device="cuda")
    y = torch.arange(1000, dtype=torch.int32, device="cuda")
    p = agg.Plan("i32", "sum", max_n=1000)
    with pytest.raises(agg.AggError):   # filter column shorter than n (beyond its allocation)
        p.run_filtered(x, agg.make_filter(y[:10]), n=2000)
    with pytest.raises(agg.AggError):   # filter in pageable host memory
        hy = np.arange(1000, dtype=np.int32)
        p.run_filtered(x, agg.make_filter(hy.ctypes.data, dtype="i32"))
    with pytest.raises(agg.AggError):   # host-source plans do not filter
        agg.Plan("i32", "sum", max_n=1000, src="pinned_host").run_filtered(x.cpu().pin_memory(), agg.make_filter(y))


def test_float_bounds_normalised_exactly(agg):
    import torch
    r = np.random.default_rng(12)
    y = np.concatenate([r.standard_normal(200_000).astype(np.float32),
                        np.array([0.1, np.float32(0.1), 1e-40, -1e-40, 0.0, -0.0, 1.0, -1.0, 3.4e38, -3.4e38,
                                  np.inf, -np.inf, np.nan], np.float32)])
    x = np.arange(y.size, dtype=np.int64)
    dx, dy = torch.from_numpy(x).to("cuda"), torch.from_numpy(y).to("cuda")
    bounds = [(0.1, 0.5), (np.float32(0.1), 1.0), (1e-41, 1e-39), (-1e-39, 0.0), (0.0, 0.0), (-np.inf, -3e38),
              (3e38, np.inf), (1e300, None), (None, -1e300), (-0.0, 1.0), (1.0, 1.0)]
    for lo, hi in bounds:
        for li in (True, False):
            for hi_inc in (True, False):
                m = mask_of(y, lo, hi, li, hi_inc)
                got = agg.Plan("i64", "sum", max_n=x.size).run_filtered(dx, agg.make_filter(dy, lo, hi, li, hi_inc))
                assert got["count"] == int(m.sum()), f"[{lo},{hi}] {li} {hi_inc}: count {got['count']} != {m.sum()}"
                assert got["i64"] == int(x[m].sum()), f"[{lo},{hi}] {li} {hi_inc}"
    with pytest.raises(agg.AggError):
        agg.Plan("i64", "sum", max_n=x.size).run_filtered(dx, agg.make_filter(dy, float("nan"), 1.0))


def test_integer_bounds_at_the_type_limits(agg):
    import torch
    y = np.array([-2**31, -2**31 + 1, -1, 0, 1, 2**31 - 2, 2**31 - 1] * 1000, np.int32)
    x = np.ones(y.size, np.int32)
    dx, dy = torch.from_numpy(x).to("cuda"), torch.from_numpy(y).to("cuda")
    for lo, hi in [(-2**63, 2**63 - 1), (-2**31, -2**31), (2**31 - 1, 2**31 - 1), (2**31, None),
                   (None, -2**31 - 1), (-2**40, 2**40), (0, 0), (2**63 - 1, None), (None, -2**63)]:
        for li in (True, False):
            for hi_inc in (True, False):
                m = mask_of(y, lo, hi, li, hi_inc)
                got = agg.Plan("i32", "count", max_n=x.size).run_filtered(dx, agg.make_filter(dy, lo, hi, li, hi_inc))
                assert got["i64"] == int(m.sum()), f"[{lo},{hi}] {li} {hi_inc}"
