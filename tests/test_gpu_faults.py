"""Error paths forced from the host (agg_fault_inject) on a real device: an
allocation failure gives AGG_E_NOMEM and leaves plans, batches, group-by
plans and servers usable; a failed shipped copy ends that request with
AGG_E_HIP, is not cached, and the other requests' results stay correct.
Nothing here reaches the device in a bad state: the failing runtime call is
never issued."""
import numpy as np
import pytest

import datagen
from aggcheck import check, same_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    yield agg
    agg.fault_inject("alloc", 0)
    agg.fault_inject("ship", 0)


def nomem(agg, make):
    agg.fault_inject("alloc", 1)
    try:
        with pytest.raises(agg.AggError) as e:
            make()
        assert e.value.code == agg.E_NOMEM
    finally:
        agg.fault_inject("alloc", 0)


def test_allocation_failures_leave_everything_usable(agg):
    import torch
    n = (1 << 22) + 9
    x = datagen.column(n, "i32", "uniform", seed=71)
    d = torch.from_numpy(x).to("cuda")
    plan = agg.Plan("i32", "sum", max_n=n)           # made before the failures
    want = plan.run(d)
    check(x, "i32", "sum", "neumaier", want)
    # plans (device and pinned-host: the second allocation of the staging ring fails)
    nomem(agg, lambda: agg.Plan("i32", "sum", max_n=n))
    agg.fault_inject("alloc", 2)
    try:
        with pytest.raises(agg.AggError) as e:
            agg.Plan("i32", "sum", max_n=n, src="pinned_host")
        assert e.value.code == agg.E_NOMEM
    finally:
        agg.fault_inject("alloc", 0)
    nomem(agg, lambda: agg.Batch([agg.BatchColumn(d, "sum")]))
    nomem(agg, lambda: agg.GroupBy("i32", "i64", "sum", max_n=n, max_groups=1 << 16))
    nomem(agg, lambda: agg.Server(hbm_budget_bytes=1 << 26, max_slots=2))
    agg.fault_inject("alloc", 3)                      # the server's third allocation (result slots)
    try:
        with pytest.raises(agg.AggError) as e:
            agg.Server(hbm_budget_bytes=1 << 26, max_slots=2)
        assert e.value.code == agg.E_NOMEM
    finally:
        agg.fault_inject("alloc", 0)
    # everything works afterwards, with the same bits
    assert same_bits(plan.run(d), want)
    assert same_bits(agg.Plan("i32", "sum", max_n=n).run(d), want)
    h = torch.from_numpy(x).pin_memory()
    assert same_bits(agg.Plan("i32", "sum", max_n=n, src="pinned_host").run(h), want)
    assert same_bits(agg.Batch([agg.BatchColumn(d, "sum")]).run()[0], want)
    keys = torch.remainder(d, 1000)
    g = agg.GroupBy("i32", "i32", "count", max_n=n, max_groups=1 << 16)
    groups = g.run(keys, d)
    assert sum(c for _, _, _, c in groups) == n
    srv = agg.Server(hbm_budget_bytes=1 << 26, max_slots=2)
    res, st, sm = srv.run([dict(ptr=h.data_ptr(), n=n, arrival_s=0.0, dtype="i32", op="sum", column_id=1)])
    srv.close()
    assert st[0]["status"] == 0 and same_bits(res[0], want)


def test_failed_shipped_copy_is_reported_and_not_cached(agg):
    import torch
    n = 3 << 22   # 48 MiB: three 16 MiB chunks
    h = torch.empty(n, dtype=torch.int32, pin_memory=True)
    datagen.fill_ptr(h.data_ptr(), n, "i32", "uniform", 72)
    x = h.numpy()
    reqs = [dict(ptr=h.data_ptr(), n=n, arrival_s=0.0, dtype="i32", op="sum", column_id=5),
            dict(ptr=h.data_ptr(), n=n, arrival_s=0.05, dtype="i32", op="max", column_id=5),
            dict(ptr=h.data_ptr(), n=n, arrival_s=0.10, dtype="i32", op="min", column_id=5)]
    srv = agg.Server(hbm_budget_bytes=1 << 28, max_slots=1, cache_shipped=True, chunk_bytes=16 << 20)
    agg.fault_inject("ship", 2)   # the first request's second chunk copy fails
    try:
        res, st, sm = srv.run(reqs)
    finally:
        agg.fault_inject("ship", 0)
    assert [s["status"] for s in st] == [agg.E_HIP, 0, 0]
    assert [s["cache_hit"] for s in st] == [0, 0, 1]     # the failed copy was not cached
    check(x, "i32", "max", "neumaier", res[1], ctx="after a failed copy")
    check(x, "i32", "min", "neumaier", res[2], ctx="cache hit after a failed copy")
    # the server keeps working
    res, st, sm = srv.run(reqs[:1])
    srv.close()
    assert st[0]["status"] == 0
    check(x, "i32", "sum", "neumaier", res[0], ctx="same server, next run")
