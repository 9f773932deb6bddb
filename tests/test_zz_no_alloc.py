"""agg_run_noalloc (the entry point for callers that cannot allocate) through
the C ABI: two calls in a row, the second on a shorter column, must give
agg_run's bits (same kernels and shape) and pass the oracle check; it takes
device and zero-copy sources, rejects the rest, and never allocates."""
import ctypes

import numpy as np
import pytest

import datagen
from aggcheck import check, same_bits

pytestmark = pytest.mark.gpu

CASES = [("i32", "sum", "neumaier"), ("i32", "count", "neumaier"), ("i64", "max", "neumaier"),
         ("i64", "avg", "neumaier"), ("f32", "sum", "neumaier"), ("f32", "avg", "f32"),
         ("f32", "sum", "f64_combine"), ("f32", "min", "neumaier")]


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    return agg


def noalloc(agg, dtype, op, prec, src, ptr, n, out):
    import torch
    L = agg.lib()
    return L.agg_run_noalloc(agg.DTYPES[dtype], agg.OPS[op], agg.PRECS[prec], agg.SRCS[src], ptr, n,
                             out.data_ptr(), torch.cuda.current_stream().cuda_stream)


def result(agg, out, dtype, op):
    import torch
    torch.cuda.synchronize()
    return agg.parse_results(out.cpu().numpy().tobytes(), [(agg.DTYPES[dtype], agg.OPS[op])])[0]


@pytest.mark.parametrize("dtype,op,prec", CASES)
def test_noalloc_equals_agg_run_twice_shrinking(agg, dtype, op, prec):
    import torch
    print(f"noalloc {dtype} {op} {prec}", flush=True)
    n1, n2 = 10_000_019, 3_000_001
    x = datagen.column(n1, dtype, "normal_outliers" if dtype == "f32" else "uniform", seed=61)
    d = torch.from_numpy(x).to("cuda")
    plan = agg.Plan(dtype, op, max_n=n1, prec=prec)
    out = torch.zeros(32, dtype=torch.uint8, device="cuda")
    for n in (n1, n2):
        assert noalloc(agg, dtype, op, prec, "device", d.data_ptr(), n, out) == agg.OK
        got = result(agg, out, dtype, op)
        want = plan.run(d, n=n)
        assert same_bits(got, want), f"{dtype} {op} {prec} n={n}: {got} != agg_run {want}"
        check(x[:n], dtype, op, prec, got, ctx=f"noalloc {dtype} {op} {prec} n={n}")
    plan.close()


def test_noalloc_zerocopy_and_empty(agg):
    import torch
    n = (1 << 20) + 3
    h = torch.empty(n, dtype=torch.int32, pin_memory=True)
    datagen.fill_ptr(h.data_ptr(), n, "i32", "uniform", 62)
    out = torch.zeros(32, dtype=torch.uint8, device="cuda")
    assert noalloc(agg, "i32", "sum", "neumaier", "zerocopy", h.data_ptr(), n, out) == agg.OK
    got = result(agg, out, "i32", "sum")
    p = agg.Plan("i32", "sum", max_n=n, src="zerocopy")
    assert same_bits(got, p.run(h))
    p.close()
    check(h.numpy(), "i32", "sum", "neumaier", got, ctx="noalloc zerocopy")
    assert noalloc(agg, "i32", "max", "neumaier", "device", 0, 0, out) == agg.OK
    r = result(agg, out, "i32", "max")
    assert r["is_null"] and r["count"] == 0


def test_noalloc_rejects_bad_arguments(agg):
    import torch
    d = torch.zeros(1024, dtype=torch.int32, device="cuda")
    out = torch.zeros(32, dtype=torch.uint8, device="cuda")
    ptr = d.data_ptr()
    assert noalloc(agg, "i32", "sum", "neumaier", "pinned_host", ptr, 1024, out) == agg.E_INVALID  # no staging
    assert noalloc(agg, "i32", "sum", "neumaier", "device", ptr + 2, 100, out) == agg.E_INVALID   # misaligned
    assert noalloc(agg, "i32", "sum", "neumaier", "device", ptr, (1 << 40) + 1, out) == agg.E_INVALID
    # past the end of the allocation (the check is against the HIP allocation's
    # extent, which for a small torch tensor is its caching-allocator segment)
    assert noalloc(agg, "i32", "sum", "neumaier", "device", ptr, 1 << 32, out) == agg.E_INVALID
    assert agg.lib().agg_run_noalloc(0, 0, 0, 0, ptr, 16, None, None) == agg.E_INVALID


def test_noalloc_allocates_nothing(agg):
    """With an allocation failure armed for the library's next allocation,
    agg_run_noalloc still succeeds, and the armed failure is still there for
    the next call that does allocate (a plan)."""
    import torch
    n = 1 << 20
    d = torch.from_numpy(datagen.column(n, "i32", "uniform", seed=63)).to("cuda")
    out = torch.zeros(32, dtype=torch.uint8, device="cuda")
    want = agg.Plan("i32", "sum", max_n=n).run(d)
    agg.fault_inject("alloc", 1)
    try:
        assert noalloc(agg, "i32", "sum", "neumaier", "device", d.data_ptr(), n, out) == agg.OK
        assert same_bits(result(agg, out, "i32", "sum"), want)
        with pytest.raises(agg.AggError) as e:
            agg.Plan("i32", "sum", max_n=n)
        assert e.value.code == agg.E_NOMEM
    finally:
        agg.fault_inject("alloc", 0)
