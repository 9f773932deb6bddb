"""GPU: aggregation of frame-of-reference + bit-packed int32 columns, from HBM
and zero-copy from pinned host memory.  Every result equals the oracle on the
raw column and agg_run on the raw column, bit for bit."""
import numpy as np
import pytest

import datagen
from aggcheck import check, same_bits

pytestmark = pytest.mark.gpu

OPS = ["sum", "min", "max", "count", "avg"]


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    return agg


def columns():
    r = np.random.default_rng(1)
    yield "uniform", datagen.column(10_000_019, "i32", "uniform", seed=1)
    yield "zipf", datagen.column(3_000_017, "i32", "zipf", seed=2)
    yield "sorted", datagen.column(3_000_017, "i32", "sorted", seed=3)
    yield "keys_sf", datagen.column(2_000_003, "i32", "uniform", seed=4, lo=1, hi=2_000_001)
    yield "full_range", r.integers(-2**31, 2**31, 1_000_003, dtype=np.int64).astype(np.int32)
    yield "constant", np.full(100_003, -5, np.int32)
    x = r.integers(-1000, 1000, 700_001).astype(np.int32)
    x[123_456], x[654_321] = -2**31, 2**31 - 1
    yield "planted_extremes", x


@pytest.mark.parametrize("name,x", list(columns()))
def test_packed_device_and_zerocopy(agg, name, x):
    import torch
    pc = agg.pack_i32(x)
    dev = pc.to("cuda")
    pin = pc.to("pinned")
    raw = torch.from_numpy(x).to("cuda")
    for op in OPS:
        ref = agg.Plan("i32", op, max_n=x.size).run(raw)
        for src, col in (("device", dev), ("zerocopy", pin)):
            got = agg.Plan("i32", op, max_n=x.size, src=src).run_packed(col)
            check(x, "i32", op, "neumaier", got, ctx=f"packed {name} {op} {src}")
            assert same_bits(ref, got), f"packed {name} {op} {src}: differs from the raw scan"


@pytest.mark.parametrize("n", [0, 1, 31, 33, 2047, 2048, 2049, 65_537, 3 * 2**20 + 5])
def test_packed_sizes_and_partial_blocks(agg, n):
    x = datagen.column(n, "i32", "uniform", seed=n + 9)
    dev = agg.pack_i32(x).to("cuda")
    for op in OPS:
        got = agg.Plan("i32", op, max_n=max(n, 1)).run_packed(dev)
        check(x, "i32", op, "neumaier", got, ctx=f"packed n={n} {op}")


def test_corrupt_block_headers_are_reported_not_read(agg):
    """A header whose payload lies outside the buffer, or whose width is
    impossible, is never read through, and the result is marked invalid
    (is_null = -1; the binding raises); the plan then works normally."""
    import torch
    x = datagen.column(100_000, "i32", "uniform", seed=5)
    pc = agg.pack_i32(x)
    good_dev = pc.to("cuda")
    bad = pc.blocks.copy()
    bad[3]["word_off"] = 10**12     # payload offset far outside the buffer
    bad[7]["bits"] = 40             # impossible width
    pc.blocks = bad
    dev = pc.to("cuda")
    pin = pc.to("pinned")
    got = agg.Plan("i32", "count", max_n=x.size).run_packed(dev)
    assert got["i64"] == x.size      # COUNT reads no block
    for op in ("sum", "min", "max", "avg"):
        for src, col in (("device", dev), ("zerocopy", pin)):
            p = agg.Plan("i32", op, max_n=x.size, src=src)
            with pytest.raises(agg.AggError) as e:
                p.run_packed(col)
            assert e.value.code == agg.E_INVALID
            out = torch.zeros(32, dtype=torch.uint8, device="cuda")
            p.enqueue_packed(col, out)
            torch.cuda.synchronize()
            assert agg.Result.from_buffer_copy(out.cpu().numpy().tobytes()).is_null == -1
            if src == "device":         # the flag was cleared: the same plan gives the right answer next
                check(x, "i32", op, "neumaier", p.run_packed(good_dev), ctx=f"after a corrupt column {op}")
            p.close()


def test_packed_rejects_wrong_plans_and_memory(agg):
    import torch
    x = datagen.column(10_000, "i32", "uniform", seed=6)
    pc = agg.pack_i32(x)
    dev = pc.to("cuda")
    with pytest.raises(agg.AggError):          # packed int32 needs an int32 plan
        agg.Plan("i64", "sum", max_n=x.size).run_packed(dev)
    with pytest.raises(agg.AggError):          # device plan given host (pageable) memory
        agg.Plan("i32", "sum", max_n=x.size).run_packed(pc)
    with pytest.raises(agg.AggError):          # zero-copy plan given device memory
        agg.Plan("i32", "sum", max_n=x.size, src="zerocopy").run_packed(dev)
    with pytest.raises(agg.AggError):          # n beyond the plan
        agg.Plan("i32", "sum", max_n=x.size - 1).run_packed(dev)


def test_packed_full_size(agg):
    import torch
    n = 1 << 30
    h = torch.empty(n, dtype=torch.int32, pin_memory=True)
    datagen.fill_ptr(h.data_ptr(), n, "i32", "uniform", 2)
    x = h.numpy()
    pc = agg.pack_i32(x)
    assert pc.nbytes < 0.67 * 4 * n
    dev, pin = pc.to("cuda"), pc.to("pinned")
    for op in ("sum", "min", "max", "avg"):
        for src, col in (("device", dev), ("zerocopy", pin)):
            got = agg.Plan("i32", op, max_n=n, src=src).run_packed(col)
            check(x, "i32", op, "neumaier", got, ctx=f"packed 2^30 {op} {src}")
