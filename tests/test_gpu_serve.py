"""GPU serving: requests admitted continuously while others run; every result
equals the oracle and, bit for bit, the same request run alone."""
import numpy as np
import pytest

import datagen
from aggcheck import check, same_bits
from datagen.serving import mean_bytes, request_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    return agg


def build_requests(agg, dtype, seed, nreq, n_max, hot_items, arena_items, rate, repeat_frac):
    import torch
    tdt = {"i32": torch.int32, "i64": torch.int64, "f32": torch.float32}[dtype]
    host = torch.empty(arena_items, dtype=tdt, pin_memory=True)
    datagen.fill_ptr(host.data_ptr(), arena_items, dtype, "uniform", seed)
    hot_h = datagen.column(hot_items, dtype, "uniform", seed=seed + 1)
    hot = torch.from_numpy(hot_h).to("cuda")
    specs = request_stream(nreq, seed=seed, n_min=10_000, n_max=n_max, rate_per_s=rate, resident_frac=0.3,
                           hot_items=hot_items, arena_items=arena_items, repeat_frac=repeat_frac)
    r = np.random.default_rng(seed)
    w = host.element_size()
    reqs, views = [], []
    for s in specs:
        prec = ["neumaier", "f32", "f64_combine"][int(r.integers(0, 3))] if dtype == "f32" else "neumaier"
        if s["resident"]:
            ptr, x = hot.data_ptr() + w * s["offset"], hot_h[s["offset"]:s["offset"] + s["n"]]
        else:
            ptr, x = host.data_ptr() + w * s["offset"], host.numpy()[s["offset"]:s["offset"] + s["n"]]
        reqs.append(dict(ptr=ptr, n=s["n"], column_id=s["column_id"], arrival_s=s["arrival_s"], dtype=dtype,
                         op=s["op"], prec=prec, resident=s["resident"]))
        views.append(x)
    return reqs, views, (host, hot)


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_mix_equals_alone_and_oracle(agg, dtype):
    n_max = 1 << 26
    cap = 55e9 / (0.7 * mean_bytes(10_000, n_max, 4))
    reqs, views, keep = build_requests(agg, dtype, seed=13, nreq=300, n_max=n_max, hot_items=1 << 27,
                                       arena_items=1 << 28, rate=0.8 * cap, repeat_frac=0.15)
    budget = 2 << 30
    srv = agg.Server(hbm_budget_bytes=budget, max_slots=8, cache_shipped=True, chunk_bytes=16 << 20)
    results, stats, summary = srv.run(reqs)
    srv.close()
    assert summary["completed"] == len(reqs) and summary["failed"] == 0
    assert summary["peak_busy_slots"] > 1, "no overlap: requests never shared the GPU"
    assert summary["peak_reserved_bytes"] <= budget
    assert summary["cache_hits"] >= 1
    lat = [s["done_s"] - s["arrival_s"] for s in stats]
    print(f"\n{dtype}: p50 {agg.percentile(lat, 50) * 1e3:.2f} ms, p99 {agg.percentile(lat, 99) * 1e3:.2f} ms, "
          f"peak slots {summary['peak_busy_slots']}, hits {summary['cache_hits']}, "
          f"shipped {summary['bytes_shipped'] / 1e9:.2f} GB in {summary['makespan_s']:.3f} s", flush=True)
    plans = {}
    for i, (q, x, got, st) in enumerate(zip(reqs, views, results, stats)):
        assert st["status"] == 0 and st["arrival_s"] <= st["admit_s"] <= st["done_s"]
        check(x, dtype, q["op"], q["prec"], got, ctx=f"request {i}")
        src = "device" if q["resident"] else "pinned_host"
        key = (q["op"], q["prec"], src)
        if key not in plans:
            plans[key] = agg.Plan(dtype, q["op"], max_n=n_max, prec=q["prec"], src=src)
        alone = plans[key].run(q["ptr"], n=q["n"])
        assert same_bits(alone, got), f"request {i} ({q['op']} {q['prec']} {src}): mix differs from alone"
    for p in plans.values():
        p.close()


def test_oversized_request_fails_without_blocking_others(agg):
    import torch
    host = torch.arange(1 << 20, dtype=torch.int32).pin_memory()
    reqs = [dict(ptr=host.data_ptr(), n=1 << 20, arrival_s=0.0, dtype="i32", op="sum", column_id=1),
            dict(ptr=host.data_ptr(), n=1 << 20, arrival_s=0.0, dtype="i32", op="max", column_id=2),
            dict(ptr=host.data_ptr(), n=1 << 18, arrival_s=0.001, dtype="i32", op="min", column_id=3)]
    srv = agg.Server(hbm_budget_bytes=2 << 20, max_slots=2)   # 2 MiB < the 4 MiB columns
    results, stats, summary = srv.run(reqs)
    srv.close()
    assert [s["status"] for s in stats] == [agg.E_NOMEM, agg.E_NOMEM, 0]
    assert results[2]["i64"] == 0 and summary["failed"] == 2


def test_serve_rejects_bad_pointers_before_running(agg):
    host = np.arange(1000, dtype=np.int32)   # pageable memory cannot be shipped
    srv = agg.Server(hbm_budget_bytes=1 << 20, max_slots=1)
    with pytest.raises(agg.AggError):
        srv.run([dict(ptr=host.ctypes.data, n=1000, arrival_s=0.0, dtype="i32", op="sum")])
    srv.close()
