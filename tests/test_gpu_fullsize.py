"""GPU parity at full workload sizes, in the launch configuration the
benchmark times (default plans): 2^30-item columns of every dtype and
distribution with every function (preloaded and from pinned host memory),
the float32 precision study with heavy cancellation, 64-bit indexing past
2^31 and 2^32 items, and the paper-shaped key-column sweep.  Every result is
checked against the CPU oracle on the full column."""
import json
import os
import sys
import time

import numpy as np
import pytest

import datagen
import oracle
from aggcheck import check, same_bits

pytestmark = pytest.mark.gpu

N = 1 << 30


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    return agg


def pinned_column(n, dtype, dist, seed, lo=0, hi=0):
    import torch
    tdt = {"i32": torch.int32, "i64": torch.int64, "f32": torch.float32}[dtype]
    h = torch.empty(n, dtype=tdt, pin_memory=True)
    datagen.fill_ptr(h.data_ptr(), n, dtype, dist, seed, lo, hi)
    return h


def free():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dist", ["uniform", "zipf", "sorted"])
@pytest.mark.parametrize("dtype", ["i32", "i64", "f32"])
def test_full_size_grid(agg, dtype, dist):
    t0 = time.time()
    seed = {"i32": 2, "i64": 5, "f32": 8}[dtype] + {"uniform": 0, "zipf": 1, "sorted": 2}[dist]
    h = pinned_column(N, dtype, dist, seed)
    x = h.numpy()
    d = h.to("cuda")
    say(f"{dtype} {dist}: generated + copied in {time.time() - t0:.1f}s")
    cases = [(op, "neumaier") for op in ("sum", "min", "max", "count", "avg")]
    if dtype == "f32":
        cases += [("sum", "f32"), ("sum", "f64_combine"), ("avg", "f32"), ("avg", "f64_combine")]
    for op, prec in cases:
        plan = agg.Plan(dtype, op, max_n=N, prec=prec)
        got = plan.run(d)
        rep = check(x, dtype, op, prec, got, ctx=f"{dtype} {dist} {op} {prec}")
        if dist == "uniform" and op in ("sum", "min"):
            hp = agg.Plan(dtype, op, max_n=N, prec=prec, src="pinned_host")
            assert same_bits(got, hp.run(h)), f"{dtype} {op}: pinned-host run differs from device run"
            hp.close()
        if rep:
            say(f"  {op} {prec}: rel {rep['rel']:.3e} kappa {rep['kappa']:.3e}")
        plan.close()
    if dist == "sorted":  # a permutation of the uniform column: integer results identical
        u = pinned_column(N, dtype, "uniform", seed)
        du = u.to("cuda")
        for op in ("sum", "min", "max"):
            if dtype == "f32" and op == "sum":
                continue
            assert same_bits(agg.Plan(dtype, op, max_n=N).run(d), agg.Plan(dtype, op, max_n=N).run(du))
        assert float(x[0]) == agg.Plan(dtype, "min", max_n=N).run(d)["value"]
        assert float(x[-1]) == agg.Plan(dtype, "max", max_n=N).run(d)["value"]
        del du, u
    del d, h
    free()
    say(f"{dtype} {dist}: done in {time.time() - t0:.1f}s")


def test_precision_study_heavy_cancellation(agg):
    """N(0,1) with 1% outliers of +-1e6: every mode within its a-priori bound,
    the compensated mode within 1e-6 relative of the exact sum."""
    h = pinned_column(N, "f32", "normal_outliers", 11)
    x = h.numpy()
    d = h.to("cuda")
    report = {}
    for prec in ("f32", "f64_combine", "neumaier"):
        got = agg.Plan("f32", "sum", max_n=N, prec=prec).run(d)
        rep = check(x, "f32", "sum", prec, got, ctx=f"precision {prec}")
        report[prec] = {"value": got["f64"], **rep}
        say(f"precision {prec}: rel {rep['rel']:.3e} abs_norm {rep['abs_norm']:.3e} kappa {rep['kappa']:.3e}")
    assert report["neumaier"]["rel"] <= 1e-6
    assert report["neumaier"]["rel"] <= report["f64_combine"]["rel"] + 1e-15
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "precision_study.json"), "w") as f:
            json.dump({"n": N, "distribution": "N(0,1) + 1% of +-1e6", "seed": 11,
                       "exact_sum": oracle.value(x, "sum"), "modes": report}, f, indent=1)
    del d, h
    free()


@pytest.mark.parametrize("n", [(1 << 31) + 5, (1 << 32) + 5])
def test_64bit_indexing(agg, n):
    import torch
    x = datagen.column(n, "i32", "uniform", seed=21)   # pageable: no power-of-two pinned block
    x[n - 1] = 2**31 - 1       # extremes at the very end: past 2^31 / 2^32 items
    x[n - 3] = -2**31
    d = torch.from_numpy(x).to("cuda")
    h = None
    for op in ("sum", "min", "max", "count", "avg"):
        got = agg.Plan("i32", op, max_n=n).run(d)
        check(x, "i32", op, "neumaier", got, ctx=f"n={n} {op}")
    del d, h
    free()


def test_paper_shaped_key_column(agg):
    """SUM over an int32 key column uniform in [1, 1e4 * SF] with 6e6 * SF rows (SF 200)."""
    sf = 200
    n = 6_000_000 * sf
    h = pinned_column(n, "i32", "uniform", 31, 1, 10_000 * sf + 1)
    x = h.numpy()
    d = h.to("cuda")
    got = agg.Plan("i32", "sum", max_n=n).run(d)
    check(x, "i32", "sum", "neumaier", got, ctx="paper-shaped SF200")
    del d, h
    free()


@pytest.mark.parametrize("card", [16, 8192, 1 << 20])
def test_groupby_full_size(agg, card):
    """Group-by as the benchmark runs it: 2^28 rows, int32 keys
    (2654435761 x) mod card of the uniform int32 column x, uniform int64 /
    float32 values, default plans for max_groups = card.  Every group's key
    and count against a host count of the keys; sampled groups' SUM / AVG /
    COUNT against the oracle over exactly that group's rows; the int64 group
    sums add up (mod 2^64) to the oracle's sum of the whole value column."""
    import torch
    n = 1 << 28
    t0 = time.time()
    xh = pinned_column(n, "i32", "uniform", 2)
    keys_d = torch.remainder(xh.to("cuda").to(torch.int64) * 2654435761, card).to(torch.int32)
    keys = keys_d.cpu().numpy()
    cnt = np.bincount(keys, minlength=card)
    present = np.flatnonzero(cnt)
    rng = np.random.default_rng(card)
    pick = rng.choice(present, size=min(22, present.size), replace=False)
    sample = np.unique(np.concatenate([present[[0, -1]], pick]))
    rows = {int(k): np.flatnonzero(keys == k) for k in sample}
    say(f"group-by {card} keys: inputs and {sample.size} sampled groups in {time.time() - t0:.1f}s")
    for vdt, op, seed in (("i64", "sum", 3), ("f32", "sum", 4), ("f32", "avg", 4), ("i32", "count", 2)):
        vh = xh if vdt == "i32" else pinned_column(n, vdt, "uniform", seed)
        v = vh.numpy()
        vd = vh.to("cuda")
        got = agg.GroupBy("i32", vdt, op, max_n=n, max_groups=card).run(keys_d, vd)
        ctx = f"group-by {card} keys {op}({vdt})"
        assert got is not None, f"{ctx}: reported overflow"
        assert [g[0] for g in got] == present.tolist(), ctx
        assert [g[3] for g in got] == cnt[present].tolist(), ctx
        by_key = {g[0]: g for g in got}
        for k, idx in rows.items():
            ref = oracle.aggregate(v[idx], op)
            g = by_key[k]
            if vdt == "f32":
                assert g[2] == ref.f64, f"{ctx}: key {k} {g[2]!r} != {ref.f64!r}"
            else:
                assert g[1] == ref.i64, f"{ctx}: key {k} {g[1]} != {ref.i64}"
        if vdt == "i64":
            total = sum(g[1] for g in got) % 2**64
            want = oracle.aggregate(v, "sum").i64 % 2**64
            assert total == want, f"{ctx}: group sums add to {total}, column sum {want}"
        del vd
        free()
        say(f"  {op}({vdt}): {len(got)} groups checked at {time.time() - t0:.1f}s")
    del keys_d
    free()


def test_batch_full_size(agg):
    """The benchmark's batch: 4096 columns, lengths log-uniform in [1e3, 1e7]
    (4.48e9 items, 23.7 GB), dtype and function drawn as the benchmark draws
    them, in the autotuned launch shape it times.  Every column's result equals
    a single agg_run of that column bit for bit and passes the oracle check."""
    import torch
    from aggcheck import check, same_bits
    t0 = time.time()
    r = np.random.default_rng(12)
    ncols = 4096
    lens = np.floor(np.exp(r.uniform(np.log(1e3), np.log(1e7), ncols))).astype(np.int64)
    dts = [["i32", "i64", "f32"][i] for i in r.integers(0, 3, ncols)]
    ops = [["sum", "min", "max", "avg"][i] for i in r.integers(0, 4, ncols)]
    host = [datagen.column(int(n), dt, "uniform", seed=1000 + i) for i, (dt, n) in enumerate(zip(dts, lens))]
    dev = [torch.from_numpy(x).to("cuda") for x in host]
    say(f"batch: {ncols} columns, {int(lens.sum())} items generated and copied in {time.time() - t0:.1f}s")
    b = agg.Batch([agg.BatchColumn(d, op) for d, op in zip(dev, ops)])
    b.autotune()
    got = b.run()
    say(f"batch: tuned {b.info()['tune']} at {time.time() - t0:.1f}s")
    plans = {}
    for i, (x, d, dt, op) in enumerate(zip(host, dev, dts, ops)):
        if (dt, op) not in plans:
            plans[(dt, op)] = agg.Plan(dt, op, max_n=int(lens.max()))
        single = plans[(dt, op)].run(d)
        assert same_bits(got[i], single), f"column {i} ({dt} {op} n={x.size}): batch != agg_run"
        check(x, dt, op, "neumaier", got[i], ctx=f"batch column {i} ({dt} {op} n={x.size})")
    for p in plans.values():
        p.close()
    b.close()
    del dev
    free()
    say(f"batch: {ncols} columns checked in {time.time() - t0:.1f}s")


def test_filter_full_size(agg):
    """The benchmark's fused-filter cells on 2^30 items (SUM(x) WHERE y < 0 for
    int32 x / float32 y, int64 x / int32 y, float32 x / int32 y, the uniform
    columns the benchmark reads): each against the oracle on x[y < 0]."""
    import torch
    t0 = time.time()
    cols = {dt: pinned_column(N, dt, "uniform", seed) for dt, seed in (("i32", 2), ("i64", 3), ("f32", 4))}
    dev = {dt: h.to("cuda") for dt, h in cols.items()}
    say(f"filter: columns generated and copied in {time.time() - t0:.1f}s")
    for vdt, fdt in (("i32", "f32"), ("i64", "i32"), ("f32", "i32")):
        filt = agg.make_filter(dev[fdt], None, 0, True, False)
        plan = agg.Plan(vdt, "sum", max_n=N)
        got = plan.run_filtered(dev[vdt], filt)
        plan.close()
        sel = cols[vdt].numpy()[cols[fdt].numpy() < 0]
        assert got["count"] == sel.size, f"SUM({vdt}) WHERE {fdt} < 0: selected {got['count']} != {sel.size}"
        check(sel, vdt, "sum", "neumaier", got, ctx=f"SUM({vdt}) WHERE {fdt} < 0")
        del sel
        say(f"  SUM({vdt}) WHERE {fdt} < 0 checked at {time.time() - t0:.1f}s")
    del dev, cols
    free()
