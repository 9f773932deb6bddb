"""GPU: group-by aggregation (agg_groupby_run) against the oracle.

The oracle sorts the row indices by key and folds each run (exact float sums
rounded once); the GPU hashes.  Groups are compared after sorting by key:
keys, counts and integer results bit for bit, float results exactly (the
GPU's float sums are exact too).  A float MIN / MAX of a group that holds
both 0.0 and -0.0 may differ in the zero's sign (both are correct: the two
compare equal), which the float comparison below allows."""
import math

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

DTS = ["i32", "i64", "f32"]
OPS = ["sum", "min", "max", "count", "avg"]
NP = {"i32": np.int32, "i64": np.int64, "f32": np.float32}


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    return agg


def same_float(a: float, b: float) -> bool:
    return (math.isnan(a) and math.isnan(b)) or a == b


def compare(got, want, ctx):
    assert got is not None, f"{ctx}: reported overflow"
    assert len(got) == len(want), f"{ctx}: {len(got)} groups != {len(want)}"
    for g, w in zip(got, want):
        assert g[0] == w[0] and g[3] == w[3], f"{ctx}: key/count {g} != {w}"
        assert g[1] == w[1], f"{ctx}: key {w[0]} i64 {g[1]} != {w[1]}"
        assert same_float(g[2], w[2]), f"{ctx}: key {w[0]} f64 {g[2]!r} != {w[2]!r}"


def make_keys(n, kdt, card, seed, dist="uniform"):
    r = np.random.default_rng(seed)
    if dist == "zipf":
        ranks = np.minimum(r.zipf(1.3, size=n), card) - 1
    else:
        ranks = r.integers(0, card, size=n)
    if kdt == "i32":
        pool = r.choice(2**32, size=card, replace=False).astype(np.int64) - 2**31
        pool[0] = -2**31
        if card > 1:
            pool[1] = 2**31 - 1
        pool = np.unique(pool)
        return pool[ranks % pool.size].astype(np.int32)
    pool = r.integers(-2**63, 2**63 - 1, size=card, dtype=np.int64)
    pool[0] = -2**63                        # the key that shares the empty-slot bit pattern
    if card > 1:
        pool[1] = 2**63 - 1
    pool = np.unique(pool)
    return pool[ranks % pool.size].astype(np.int64)


def make_vals(n, vdt, seed):
    if vdt == "f32":
        r = np.random.default_rng(seed)
        return (r.standard_normal(n) * np.exp2(r.integers(-40, 41, size=n))).astype(np.float32)
    return datagen.column(n, vdt, "uniform", seed=seed)


def run_case(agg, keys, vals, op, max_groups, ctx):
    import torch
    kdt = {np.dtype(np.int32): "i32", np.dtype(np.int64): "i64"}[keys.dtype]
    vdt = {np.dtype(np.int32): "i32", np.dtype(np.int64): "i64", np.dtype(np.float32): "f32"}[vals.dtype]
    g = agg.GroupBy(kdt, vdt, op, max_n=max(keys.size, 1), max_groups=max_groups)
    got = g.run(torch.from_numpy(keys).to("cuda"), torch.from_numpy(vals).to("cuda"))
    compare(got, oracle.groupby(keys, vals, op), ctx)


@pytest.mark.parametrize("vdt", DTS)
@pytest.mark.parametrize("kdt", ["i32", "i64"])
def test_groupby_matches_oracle(agg, kdt, vdt):
    n = 200_003
    for card in (1, 16, 1000, 50_000):
        keys = make_keys(n, kdt, card, seed=card)
        vals = make_vals(n, vdt, seed=card + 1)
        for op in OPS:
            run_case(agg, keys, vals, op, max_groups=max(card, 1), ctx=f"{kdt}/{vdt} card={card} {op}")


@pytest.mark.parametrize("vdt", DTS)
def test_groupby_skewed_keys(agg, vdt):
    """Zipf-distributed keys: a few groups take most rows (LDS contention)."""
    n = 1_000_003
    keys = make_keys(n, "i64", 5000, seed=21, dist="zipf")
    vals = make_vals(n, vdt, seed=22)
    for op in OPS:
        run_case(agg, keys, vals, op, max_groups=5000, ctx=f"zipf {vdt} {op}")


def test_groupby_many_groups(agg):
    """More distinct keys than any workgroup's LDS table: the global table path."""
    n = 3_000_017
    r = np.random.default_rng(5)
    keys = r.integers(-2**40, 2**40, size=n, dtype=np.int64) // 4
    keys = keys % 1_000_003
    vals = make_vals(n, "f32", seed=6)
    for op in ("sum", "count", "max"):
        run_case(agg, keys, vals, op, max_groups=1_000_003, ctx=f"many groups {op}")
    vals_i = make_vals(n, "i64", seed=7)
    run_case(agg, keys, vals_i, "sum", max_groups=1_000_003, ctx="many groups i64 sum")


def test_groupby_float_specials(agg):
    import torch
    keys = np.repeat(np.arange(6, dtype=np.int32), 1000)
    vals = np.ones(keys.size, np.float32)
    vals[0] = np.nan                       # group 0: NaN
    vals[1000] = np.inf                    # group 1: +inf
    vals[2000] = -np.inf                   # group 2: -inf
    vals[3000], vals[3001] = np.inf, -np.inf   # group 3: NaN
    vals[4000:5000] = np.nan               # group 4: every item NaN -> MIN / MAX NaN
    vals[5000:5500], vals[5500:] = 3.4e38, 3.4e38   # group 5: sum beyond float range, finite in double
    for op in OPS:
        run_case(agg, keys, vals, op, max_groups=6, ctx=f"specials {op}")
    # signed zeros: MIN / MAX compare equal to the oracle's whichever zero they pick
    z = np.array([0.0, -0.0] * 500, np.float32)
    g = agg.GroupBy("i32", "f32", "min", max_n=z.size, max_groups=1)
    got = g.run(torch.zeros(z.size, dtype=torch.int32, device="cuda"), torch.from_numpy(z).to("cuda"))
    assert got[0][2] == 0.0 and got[0][3] == z.size


def test_groupby_float_sum_is_exact(agg):
    """Cancelling float sums: the exact value rounded once, whatever the order."""
    n = 400_000
    r = np.random.default_rng(9)
    keys = r.integers(0, 7, size=n).astype(np.int32)
    x = (r.standard_normal(n // 2) * np.exp2(r.integers(-60, 61, size=n // 2))).astype(np.float32)
    vals = np.concatenate([x, -x])
    vals[::1001] = np.float32(1e-30)
    keys = keys[r.permutation(n)]
    run_case(agg, keys, vals, "sum", max_groups=7, ctx="cancelling sums")
    run_case(agg, keys, vals, "avg", max_groups=7, ctx="cancelling avg")


def test_groupby_float_sum_full_exponent_range(agg):
    """Float sums over every exponent, subnormals included: an LDS slot keeps
    the middle digits only, and rows whose digits fall outside them (tiny and
    huge magnitudes) take the global table; both halves must add up exactly,
    on the direct and on the partitioned path."""
    n = 300_007
    r = np.random.default_rng(17)
    e = r.integers(-149, 128, size=n)
    m = 1.0 + r.random(n)
    vals = (np.where(r.random(n) < 0.5, -1.0, 1.0) * np.ldexp(m, e)).astype(np.float32)
    vals[~np.isfinite(vals)] = np.float32(3.0e38)
    vals[::97] = np.float32(0.0)
    assert (np.abs(vals[vals != 0]) < 2.0**-94).any() and (np.abs(vals) >= 2.0**98).any()
    for card, mg in ((5, 5), (5, 100_000), (3000, 3000)):
        keys = r.integers(0, card, size=n).astype(np.int32)
        for op in ("sum", "avg"):
            run_case(agg, keys, vals, op, max_groups=mg, ctx=f"exponent range card={card} plan={mg} {op}")


def test_groupby_overflow_and_limits(agg):
    import torch
    keys = np.arange(1000, dtype=np.int64) * 7919
    vals = np.ones(1000, np.int32)
    dk, dv = torch.from_numpy(keys).to("cuda"), torch.from_numpy(vals).to("cuda")
    assert agg.GroupBy("i64", "i32", "sum", max_n=1000, max_groups=999).run(dk, dv) is None
    assert agg.GroupBy("i64", "i32", "sum", max_n=1000, max_groups=400).run(dk, dv) is None
    assert agg.GroupBy("i64", "i32", "sum", max_n=1000, max_groups=10).run(dk, dv) is None
    got = agg.GroupBy("i64", "i32", "sum", max_n=1000, max_groups=1000).run(dk, dv)
    assert [g[0] for g in got] == sorted(keys.tolist()) and all(g[1] == 1 for g in got)


def test_groupby_empty_and_reuse(agg):
    import torch
    g = agg.GroupBy("i32", "i64", "sum", max_n=100_000, max_groups=100)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    assert g.run(e, torch.empty(0, dtype=torch.int64, device="cuda")) == []
    for n, seed in ((100_000, 1), (5000, 2), (1, 3), (0, 4), (77_777, 5)):
        keys = make_keys(n, "i32", 100, seed=seed) if n else np.zeros(0, np.int32)
        vals = make_vals(n, "i64", seed=seed)
        got = g.run(torch.from_numpy(keys).to("cuda"), torch.from_numpy(vals).to("cuda"), n=n)
        compare(got, oracle.groupby(keys, vals, "sum"), f"reuse n={n}")


def test_groupby_errors(agg):
    import torch
    with pytest.raises(agg.AggError):
        agg.GroupBy("f32", "i32", "sum", max_n=10, max_groups=10)     # float keys
    with pytest.raises(agg.AggError):
        agg.GroupBy("i32", "i32", "sum", max_n=10, max_groups=0)
    with pytest.raises(agg.AggError):
        agg.GroupBy("i32", "f32", "sum", max_n=2**31 + 1, max_groups=10)   # float digit headroom
    g = agg.GroupBy("i32", "i32", "sum", max_n=100, max_groups=10)
    k = torch.zeros(200, dtype=torch.int32, device="cuda")
    with pytest.raises(agg.AggError):
        g.run(k, k, n=200)                                                    # beyond max_n
    with pytest.raises(agg.AggError):
        g.run(np.zeros(10, np.int32).ctypes.data, k, n=10)                    # pageable host keys
    raw = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(agg.AggError):
        g.run(raw.data_ptr() + 2, k, n=10)                                    # keys not 4-byte aligned
    g64 = agg.GroupBy("i64", "i64", "sum", max_n=100, max_groups=10)
    k64 = torch.zeros(100, dtype=torch.int64, device="cuda")
    with pytest.raises(agg.AggError):
        g64.run(k64, raw.data_ptr() + 4, n=10)                               # values not 8-byte aligned
    got = g.run(k, k, n=100)                                                  # the plan still works
    assert got == [(0, 0, 0.0, 100)]
    g64.close()
    g.close()


def test_groupby_partitioned_with_few_actual_groups(agg):
    """A plan sized for many groups (partitioned path) on an input with few."""
    n = 500_009
    keys = make_keys(n, "i64", 37, seed=31)
    for vdt in DTS:
        vals = make_vals(n, vdt, seed=32)
        for op in ("sum", "min", "count"):
            run_case(agg, keys, vals, op, max_groups=100_000, ctx=f"few groups, big plan {vdt} {op}")
    # more partitions than the scatter takes: several aggregation passes per partition
    many = make_keys(n, "i32", 20_000, seed=33)
    for vdt in ("f32", "i64"):
        for op in ("sum", "min", "count"):
            run_case(agg, many, make_vals(n, vdt, seed=34), op, max_groups=6_000_000, ctx=f"sub-partitions {vdt} {op}")
    wide = make_keys(n, "i64", 150_000, seed=35)      # 8 passes per partition for float sums
    run_case(agg, wide, make_vals(n, "f32", seed=36), "sum", max_groups=8_000_000, ctx="8 sub-partitions f32 sum")
    run_case(agg, wide, make_vals(n, "i32", seed=37), "avg", max_groups=30_000_000, ctx="8 sub-partitions i32 avg")


@pytest.mark.parametrize("kdt,vdt,op,half", [
    ("i32", "i64", "sum", 4096), ("i32", "i32", "count", 8192), ("i32", "f32", "sum", 512),
    ("i64", "i64", "max", 2048), ("i64", "i32", "count", 4096), ("i64", "f32", "avg", 512)])
def test_groupby_path_boundaries(agg, kdt, vdt, op, half):
    """Plans at half an LDS table (the last one-pass direct plan), one group
    past it (two direct passes; COUNT: partitioned), at a whole table (the
    last two-pass plan) and one past that (the first partitioned plan), each
    with exactly max_groups distinct keys."""
    n = 300_007
    for groups in (half, half + 1, 2 * half, 2 * half + 1):
        keys = make_keys(n, kdt, groups, seed=groups)
        assert np.unique(keys).size == groups
        vals = make_vals(n, vdt, seed=groups + 7)
        run_case(agg, keys, vals, op, max_groups=groups, ctx=f"{kdt}/{vdt} {op} {groups} groups")


def test_groupby_result_independent_of_path(agg):
    """The same rows through every path -- one direct pass, two direct passes,
    partitioned, partitioned with sub-partition passes -- give the same groups
    bit for bit (float sums are exact, so no path's row order shows)."""
    import torch
    n = 400_009
    keys = make_keys(n, "i32", 300, seed=41)
    dk = torch.from_numpy(keys).to("cuda")
    for vdt, op in (("f32", "sum"), ("f32", "avg"), ("i64", "sum"), ("f32", "max")):
        vals = make_vals(n, vdt, seed=42)
        dv = torch.from_numpy(vals).to("cuda")
        want = oracle.groupby(keys, vals, op)
        first = None
        for mg in (300, 600, 5000, 100_000, 6_000_000):
            got = agg.GroupBy("i32", vdt, op, max_n=n, max_groups=mg).run(dk, dv)
            compare(got, want, f"{vdt} {op} max_groups={mg}")
            if first is None:
                first = got
            assert got == first, f"{vdt} {op}: max_groups={mg} differs from max_groups=300"


def test_groupby_plans_on_concurrent_streams(agg):
    """Four plans (direct, two-pass, partitioned, sub-partition passes) run
    at once on four streams, twice each, share no state: every result equals
    the oracle's."""
    import torch
    n = 250_007
    cases = []
    for i, (card, mg, vdt, op) in enumerate(((100, 100, "i64", "sum"), (1500, 2000, "f32", "sum"),
                                             (20_000, 20_000, "i32", "count"), (30_000, 6_000_000, "f32", "avg"))):
        keys = make_keys(n, "i32", card, seed=60 + i)
        vals = make_vals(n, vdt, seed=70 + i)
        g = agg.GroupBy("i32", vdt, op, max_n=n, max_groups=mg)
        out = torch.empty(mg * agg.GROUP_BYTES, dtype=torch.uint8, device="cuda")
        ng = torch.zeros(1, dtype=torch.int64, device="cuda")
        cases.append((g, torch.from_numpy(keys).to("cuda"), torch.from_numpy(vals).to("cuda"), out, ng,
                      torch.cuda.Stream(), oracle.groupby(keys, vals, op), f"{vdt} {op} plan {mg}"))
    torch.cuda.synchronize()
    for _ in range(2):
        for g, dk, dv, out, ng, st, _, _ in cases:
            g.enqueue(dk, dv, out, ng, stream=st)
    torch.cuda.synchronize()
    for g, dk, dv, out, ng, st, want, ctx in cases:
        k = int(ng.item())
        raw = out[:k * agg.GROUP_BYTES].cpu().numpy().tobytes()
        got = sorted(((x.key, x.i64, x.f64, x.count) for x in
                      (agg.Group.from_buffer_copy(raw, i * agg.GROUP_BYTES) for i in range(k))), key=lambda t: t[0])
        compare(got, want, ctx)
        g.close()


@pytest.mark.parametrize("kdt", ["i32", "i64"])
def test_groupby_single_marker_key(agg, kdt):
    """Every row has the key whose bit pattern marks an empty slot (INT32_MIN /
    INT64_MIN): one group, through the direct path, the partitioned path (all
    rows in one partition) and sub-partition passes."""
    n = 200_003
    keys = np.full(n, np.iinfo(NP[kdt]).min, dtype=NP[kdt])
    for vdt, op in (("i64", "sum"), ("f32", "sum"), ("i32", "count")):
        vals = make_vals(n, vdt, seed=81)
        for mg in (1, 100_000, 6_000_000):
            run_case(agg, keys, vals, op, max_groups=mg, ctx=f"marker key {kdt} {vdt} {op} plan {mg}")


def test_groupby_multi_chunk_closed_form(agg):
    """More rows than one partitioning chunk (2^28), more groups than the
    direct path takes: per-key sums with closed forms."""
    import math
    import torch
    n = (1 << 28) + 4099
    card = 10007
    idx = torch.arange(n, dtype=torch.int64, device="cuda")
    keys = (idx % card).to(torch.int32)
    r = np.arange(card, dtype=np.int64)
    cnt = n // card + (r < n % card)                          # rows r, r + card, r + 2 card, ...
    got = agg.GroupBy("i32", "i64", "sum", max_n=n, max_groups=card).run(keys, idx)
    want_sum = r * cnt + card * cnt * (cnt - 1) // 2          # sum of r + card*j for j < cnt[r]
    assert [g[0] for g in got] == list(range(card))
    assert [g[3] for g in got] == cnt.tolist()
    assert [g[1] for g in got] == want_sum.tolist()
    vf = ((idx % 7) - 3).to(torch.float32)
    del idx
    got = agg.GroupBy("i32", "f32", "sum", max_n=n, max_groups=card).run(keys, vf)
    # (r + card*j) mod 7 runs through all residues every 7 steps of j (card is
    # prime to 7) and those 7 values of x - 3 sum to 0: only the last cnt mod 7 count
    assert math.gcd(card, 7) == 1
    want_f = [float(sum((rr + card * j) % 7 - 3 for j in range(c % 7))) for rr, c in zip(r.tolist(), cnt.tolist())]
    assert [g[2] for g in got] == want_f


def test_groupby_float_sum_rounding_cases(agg):
    """Group sums that land exactly between two doubles (ties to even), just
    above a tie (sticky bit), and ones that need every digit."""
    import torch
    t = np.float32(2.0**53)
    groups = {0: [t, 1.0], 1: [t, 3.0], 2: [t, 1.0, 2.0**-20], 3: [t, -1.0], 4: [2.0**-149] * 3,
              5: [3.4e38, 3.4e38, -3.4e38, 1e-45], 6: [1.0, 2.0**-24, 2.0**-24], 7: [-t, -1.0]}
    want = {0: 2.0**53, 1: 2.0**53 + 4, 2: 2.0**53 + 2, 3: 2.0**53 - 1, 4: 3 * 2.0**-149,
            5: float(np.float32(3.4e38)) + 2.0**-149, 6: 1.0 + 2.0**-23, 7: -2.0**53}
    keys = np.concatenate([np.full(len(v), k, np.int32) for k, v in groups.items()])
    vals = np.concatenate([np.array(v, np.float32) for v in groups.values()])
    g = agg.GroupBy("i32", "f32", "sum", max_n=keys.size, max_groups=8)
    got = g.run(torch.from_numpy(keys).to("cuda"), torch.from_numpy(vals).to("cuda"))
    assert [x[2] for x in got] == [want[k] for k in sorted(want)]
    compare(got, oracle.groupby(keys, vals, "sum"), "rounding cases")


def test_groupby_declared_max_groups_does_not_change_groups(agg):
    """The declared max_groups picks the path (direct, direct in two passes,
    partitioned); over the same 12 groups every choice gives the same groups
    bit for bit, and the oracle's, including the marker key and float values
    outside the LDS digits."""
    import torch
    n = 300_007
    for kdt in ("i32", "i64"):
        keys = make_keys(n, kdt, 12, seed=92)   # the pool holds the marker key (INT_MIN)
        dk = torch.from_numpy(keys).to("cuda")
        for vdt, op in (("f32", "sum"), ("i64", "sum"), ("i32", "min"), ("f32", "max"), ("i32", "count")):
            vals = make_vals(n, vdt, seed=93)
            if vdt == "f32":
                vals[::777] = np.float32(2.0 ** 100)
                vals[::555] = np.float32(2.0 ** -120)
            dv = torch.from_numpy(vals).to("cuda")
            want = oracle.groupby(keys, vals, op)
            assert len(want) == 12
            first = None
            for mg in (12, 16, 17, 5000, 100_000, 6_000_000):
                got = agg.GroupBy(kdt, vdt, op, max_n=n, max_groups=mg).run(dk, dv)
                compare(got, want, f"{kdt} {vdt} {op} max_groups={mg}")
                if first is None:
                    first = got
                assert got == first, f"{kdt} {vdt} {op}: max_groups={mg} differs from max_groups=12"
