"""GPU parity: the HIP scan through the C ABI against the CPU oracle.

Sizes span one partial wave load up to hundreds of segments, with ragged
tails; every dtype, function and float precision mode; aligned and unaligned
column addresses; pinned-host (chunked) and zero-copy sources; many launch
configurations (which must not change a bit); repeated runs; and the error
paths of agg_run on a real device.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle
from aggcheck import check, same_bits

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 3, 4, 5, 15, 16, 17, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4095, 4096,
         4097, 16383, 65539, 2**20, 2**20 + 13, 3 * 2**20 + 5, 10_000_019]
CASES = [("i32", op, "neumaier") for op in ("sum", "min", "max", "count", "avg")] + \
        [("i64", op, "neumaier") for op in ("sum", "min", "max", "count", "avg")] + \
        [("f32", op, "neumaier") for op in ("min", "max", "count")] + \
        [("f32", op, prec) for op in ("sum", "avg") for prec in ("neumaier", "f32", "f64_combine")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    assert agg.device_info(0)["arch"].startswith("gfx950")
    return agg


def tdev(x: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def column(dtype: str, n: int, seed: int, kind: str = "uniform") -> np.ndarray:
    if kind == "wide" and dtype == "f32":   # heavy cancellation, magnitudes 2^-20 .. 2^20
        r = np.random.default_rng(seed)
        return (r.standard_normal(n) * np.exp2(r.integers(-20, 21, size=n))).astype(np.float32)
    return datagen.column(n, dtype, kind if kind != "wide" else "uniform", seed=seed)


@pytest.mark.parametrize("dtype,op,prec", CASES)
def test_parity_all_sizes(agg, dtype, op, prec):
    big = column(dtype, max(SIZES), seed=100 + len(op), kind="wide" if dtype == "f32" else "uniform")
    # planted extremes in the middle of the longer columns
    if dtype != "f32":
        lo, hi = np.iinfo(big.dtype).min, np.iinfo(big.dtype).max
        big[777_777] = lo
        big[5_555_555] = hi
    d = tdev(big)
    plan = agg.Plan(dtype, op, max_n=big.size, prec=prec)
    say(f"parity {dtype} {op} {prec}")
    for n in SIZES:
        got = plan.run(d[:n] if n else d[:0], n=n)
        check(big[:n], dtype, op, prec, got, ctx=f"{dtype} {op} {prec} n={n}")
    plan.close()


@pytest.mark.parametrize("dtype", ["i32", "i64", "f32"])
@pytest.mark.parametrize("dist", ["zipf", "sorted"])
def test_parity_distributions(agg, dtype, dist):
    n = 5_000_011
    x = datagen.column(n, dtype, dist, seed=7)
    d = tdev(x)
    for op in ("sum", "min", "max", "avg"):
        got = agg.Plan(dtype, op, max_n=n).run(d)
        check(x, dtype, op, "neumaier", got, ctx=f"{dtype} {dist} {op}")


@pytest.mark.parametrize("dtype", ["i32", "i64", "f32"])
def test_unaligned_addresses_match_aligned_copy(agg, dtype):
    import torch
    x = column(dtype, 3_000_017, seed=31, kind="wide")
    d = tdev(x)
    for op, prec in [("sum", "neumaier"), ("sum", "f32"), ("min", "neumaier"), ("max", "neumaier"),
                     ("avg", "f64_combine")]:
        if dtype != "f32" and prec != "neumaier":
            continue
        plan = agg.Plan(dtype, op, max_n=x.size, prec=prec)
        for off in (1, 2, 3):
            if (off * x.itemsize) % 16 == 0:
                continue
            n = x.size - off - 5
            view = d[off:off + n]
            assert view.data_ptr() % 16 != 0
            got = plan.run(view)
            check(x[off:off + n], dtype, op, prec, got, ctx=f"unaligned {dtype} {op} off={off}")
            copy = torch.empty(n + 64, dtype=d.dtype, device="cuda")[:n]
            copy.copy_(view)
            assert copy.data_ptr() % 16 == 0
            assert same_bits(got, plan.run(copy)), f"{dtype} {op} {prec} off={off}: aligned copy differs"


def test_launch_parameters_do_not_change_bits(agg):
    x = column("f32", 7_000_003, seed=5, kind="wide")
    d = tdev(x)
    tunes = [dict(unroll=u, waves_per_block=w, blocks_per_cu=b, nontemporal=nt)
             for u, w, b, nt in [(4, 4, 1, 0), (8, 4, 8, 1), (16, 4, 2, 1), (8, 8, 4, 0), (16, 16, 1, 1),
                                 (4, 16, 32, 0), (8, 4, 32, 1)]]
    for op, prec in [("sum", "neumaier"), ("sum", "f32"), ("sum", "f64_combine"), ("min", "neumaier")]:
        ref = None
        for t in tunes:
            got = agg.Plan("f32", op, max_n=x.size, prec=prec, tune=agg.make_tune(**t)).run(d)
            if ref is None:
                ref = got
                check(x, "f32", op, prec, got, ctx=f"tune {t}")
            assert same_bits(ref, got), f"{op} {prec}: tune {t} changed the result"
    for dtype in ("i32", "i64"):
        xi = column(dtype, 4_000_037, seed=6)
        di = tdev(xi)
        for t in tunes:
            got = agg.Plan(dtype, "sum", max_n=xi.size, tune=agg.make_tune(**t)).run(di)
            check(xi, dtype, "sum", "neumaier", got, ctx=f"tune {t}")


def test_repeated_runs_are_bitwise_identical(agg):
    x = column("f32", 10_000_019, seed=9, kind="wide")
    d = tdev(x)
    for prec in ("neumaier", "f32", "f64_combine"):
        plan = agg.Plan("f32", "sum", max_n=x.size, prec=prec)
        first = plan.run(d)
        for _ in range(10):
            assert same_bits(first, plan.run(d))


@pytest.mark.parametrize("dtype,op,prec", [("i64", "sum", "neumaier"), ("i32", "min", "neumaier"),
                                           ("f32", "sum", "neumaier"), ("f32", "avg", "f64_combine")])
def test_back_to_back_calls_read_their_own_partials(agg, dtype, op, prec):
    """One plan, 96 calls queued with no synchronisation between them, cycling
    over three columns and four lengths, under two launch shapes (the second
    with up to 8192 workgroups): every result is its own column's.  Small
    columns take one launch whose last workgroup merges partials that other
    workgroups, on other XCDs, stored in the same launch over the previous
    call's partials, and the plan's finished-workgroup counter must be zero
    again after every launch; 2^22 + 7 items take two launches, 2^22 int32 /
    float32 items (1024 partials on 256 workgroups) one, at the boundary."""
    import torch
    n = (1 << 22) + 7
    cols = [column(dtype, n, seed=300 + i, kind="wide" if dtype == "f32" else "uniform") for i in range(3)]
    ds = [tdev(c) for c in cols]
    lens = [n, 1 << 22, (1 << 18) + 7, 1000]
    calls = 96
    for t in (None, dict(unroll=8, waves_per_block=4, blocks_per_cu=32, nontemporal=1)):
        kw = {"tune": agg.make_tune(**t)} if t else {}
        plan = agg.Plan(dtype, op, max_n=n, prec=prec, **kw)
        out = torch.zeros((calls, agg.RESULT_BYTES), dtype=torch.uint8, device="cuda")
        say(f"back-to-back {dtype} {op} {prec} tune {t}")
        for k in range(calls):
            plan.enqueue(ds[k % 3], out[k], n=lens[(k // 3) % 4])
        torch.cuda.synchronize()
        got = agg.parse_results(out.cpu().numpy().tobytes(), [(plan.dtype, plan.op)] * calls)
        first = {}
        for k in range(calls):
            key = (k % 3, (k // 3) % 4)
            if key not in first:
                first[key] = got[k]
                check(cols[key[0]][:lens[key[1]]], dtype, op, prec, got[k], ctx=f"call {k} tune {t}")
            else:
                assert same_bits(first[key], got[k]), f"call {k} (column {key[0]}, length {key[1]}) tune {t}"
        plan.close()


@pytest.mark.parametrize("src", ["pinned_host", "zerocopy"])
@pytest.mark.parametrize("dtype", ["i32", "i64", "f32"])
def test_host_sources_match_device(agg, src, dtype):
    import torch
    n = 9_000_007
    x = column(dtype, n, seed=41, kind="wide")
    host = torch.from_numpy(x).pin_memory()
    d = host.to("cuda")
    for op, prec in [("sum", "neumaier"), ("sum", "f32"), ("min", "neumaier"), ("avg", "f64_combine"),
                     ("count", "neumaier")]:
        if dtype != "f32" and prec != "neumaier":
            continue
        ref = agg.Plan(dtype, op, max_n=n, prec=prec).run(d)
        for tune in (None, agg.make_tune(chunk_bytes=1 << 20, staging_depth=2),
                     agg.make_tune(chunk_bytes=3 << 20, staging_depth=4, unroll=4)):
            plan = agg.Plan(dtype, op, max_n=n, prec=prec, src=src, tune=tune)
            for m in (n, n - 12345, 100, 0):
                got = plan.run(host[:m] if m else host[:0], n=m)
                if m == n:
                    assert same_bits(ref, got), f"{src} {dtype} {op} {prec}: differs from device"
                check(x[:m], dtype, op, prec, got, ctx=f"{src} {dtype} {op} n={m}")
            plan.close()


def test_result_written_to_device_memory(agg):
    import torch
    x = column("i64", 1_000_003, seed=3)
    d = tdev(x)
    plan = agg.Plan("i64", "sum", max_n=x.size)
    out = torch.zeros(32, dtype=torch.uint8, device="cuda")
    plan.enqueue(d, out)
    torch.cuda.synchronize()
    r = agg.parse_results(out.cpu().numpy().tobytes(), [(agg.I64, agg.SUM)])[0]
    assert r["i64"] == oracle.value(x, "sum")


def test_errors_on_device(agg):
    import torch
    L = agg.lib()
    x = tdev(np.arange(1000, dtype=np.int32))
    plan = agg.Plan("i32", "sum", max_n=1 << 20)
    out = torch.zeros(32, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.agg_run(plan._h, x.data_ptr() + 1, 10, out.data_ptr(), s) == agg.E_INVALID   # misaligned
    assert L.agg_run(plan._h, x.data_ptr(), (1 << 20) + 1, out.data_ptr(), s) == agg.E_INVALID  # > max_n
    host = np.arange(1000, dtype=np.int32)                                               # pageable host
    assert L.agg_run(plan._h, host.ctypes.data, 1000, out.data_ptr(), s) == agg.E_INVALID
    pinned = torch.arange(1000, dtype=torch.int32).pin_memory()                          # wrong source
    assert L.agg_run(plan._h, pinned.data_ptr(), 1000, out.data_ptr(), s) == agg.E_INVALID
    big = agg.Plan("i32", "sum", max_n=1 << 34)
    assert L.agg_run(big._h, x.data_ptr(), 1 << 33, out.data_ptr(), s) == agg.E_INVALID  # beyond allocation
    hp = agg.Plan("i32", "sum", max_n=1 << 20, src="pinned_host")
    assert L.agg_run(hp._h, x.data_ptr(), 1000, out.data_ptr(), s) == agg.E_INVALID     # device ptr to host plan
    # the plan still works after rejected calls
    torch.cuda.synchronize()
    assert plan.run(x)["i64"] == 999 * 1000 // 2


SHAPE_SIZES = [1, 5, 255, 256, 257, 1000, 1023, 1025, 4096 + 3, 65536 + 17, (1 << 20) + 7, (3 << 20) + 5,
               10_000_019]


@pytest.mark.parametrize("prec", ["neumaier", "f64_combine", "f32"])
@pytest.mark.parametrize("dist", ["normal_outliers", "uniform"])
def test_float_sum_follows_canonical_shape_bit_for_bit(agg, prec, dist):
    """Float SUM bits equal the step-by-step numpy model of the documented
    canonical shape (lane folds with renormalisation every 4 rounds, merge
    trees, double combine), for aligned and unaligned addresses, in a batch
    and through an always-true filter."""
    import torch
    import shape_model as sm
    big = datagen.column(max(SHAPE_SIZES) + 1, "f32", dist, seed=41)
    d = tdev(big)
    plan = agg.Plan("f32", "sum", max_n=big.size, prec=prec)
    ones = torch.ones(big.size, dtype=torch.int32, device="cuda")
    always = agg.make_filter(ones, 1, 1, True, True)
    say(f"shape {prec} {dist}")
    for n in SHAPE_SIZES:
        want = sm.model_sum(big[:n], prec)
        got = plan.run(d[:n], n=n)["f64"]
        assert got == want, f"{prec} {dist} n={n}: GPU {got!r} != model {want!r}"
        got_u = plan.run(d[1:n + 1], n=n)["f64"]   # 4-byte aligned only: the item-wise path
        assert got_u == sm.model_sum(big[1:n + 1], prec), f"{prec} {dist} n={n}: unaligned"
        got_f = plan.run_filtered(d[:n], always, n=n)["f64"]
        assert got_f == want, f"{prec} {dist} n={n}: filtered {got_f!r} != {want!r}"
    cols = [agg.BatchColumn(d[:n], "sum", prec=prec) for n in SHAPE_SIZES[-4:]]
    b = agg.Batch(cols)
    for n, r in zip(SHAPE_SIZES[-4:], b.run()):
        assert r["f64"] == sm.model_sum(big[:n], prec), f"batch {prec} n={n}"
    b.close()
    plan.close()
