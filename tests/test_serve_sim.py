"""The serving scheduler's host logic, on the CPU with the simulated executor:
admission order, slot and HBM-budget limits, continuous admission (overlap),
the resident cache with LRU eviction, and requests that can never fit."""
import numpy as np
import pytest

import paper_2606_10030_amd as agg
from datagen.serving import request_stream

GB = 1e9


def reqs_of(specs, dtype="i32", base=1 << 20):
    out = []
    for s in specs:
        out.append(dict(ptr=base + 4 * s.get("offset", 0), n=s["n"], arrival_s=s["arrival_s"], dtype=dtype,
                        op=s.get("op", "sum"), resident=s.get("resident", False),
                        column_id=s.get("column_id", 0)))
    return out


def test_all_complete_within_slot_and_budget_limits():
    specs = request_stream(500, seed=1, n_min=10_000, n_max=1 << 28, rate_per_s=400.0,
                           resident_frac=0.3, hot_items=1 << 28, arena_items=1 << 28)
    reqs = reqs_of(specs)
    budget = 3 << 30
    st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=budget, max_slots=4, cache_shipped=False)
    assert sm["completed"] == 500 and sm["failed"] == 0
    assert sm["peak_busy_slots"] <= 4
    assert sm["peak_reserved_bytes"] <= budget
    assert sm["peak_busy_slots"] > 1                      # continuous admission: work overlapped
    for s in st:
        assert s["status"] == 0 and s["arrival_s"] <= s["admit_s"] <= s["done_s"]
    shipped = sum(4 * q["n"] for q in specs if not q["resident"])
    assert sm["bytes_shipped"] == shipped
    assert sm["bytes_scanned"] == sum(4 * q["n"] for q in specs)


def test_one_slot_is_fifo_and_serialised():
    reqs = reqs_of([dict(n=1 << 20, arrival_s=0.001 * i) for i in range(20)])
    st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=1 << 30, max_slots=1, pcie_gbs=10.0, hbm_gbs=1000.0,
                                launch_s=0.0)
    admits = [s["admit_s"] for s in st]
    assert admits == sorted(admits)
    for a, b in zip(st, st[1:]):
        assert b["admit_s"] >= a["done_s"] - 1e-12          # no overlap with one slot
    # service time of a shipped request = copy at 10 GB/s (the scan overlaps it)
    assert abs((st[0]["done_s"] - st[0]["admit_s"]) - (4 << 20) / 10e9) < 1e-9


def test_budget_blocks_shipped_but_not_resident_requests():
    big = dict(n=(3 << 30) // 4, arrival_s=0.0)              # 3 GiB shipped
    reqs = reqs_of([big, dict(big, arrival_s=0.0001),          # second big one must wait for memory
                    dict(n=1000, arrival_s=0.0002, resident=True),
                    dict(n=1000, arrival_s=0.0003, resident=True)])
    st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=4 << 30, max_slots=4, cache_shipped=False,
                                pcie_gbs=50.0)
    assert st[1]["admit_s"] >= st[0]["done_s"] - 1e-12         # waited for the first to free memory
    assert st[2]["admit_s"] < st[0]["done_s"] and st[3]["admit_s"] < st[0]["done_s"]  # resident bypass
    assert sm["peak_reserved_bytes"] <= 4 << 30


def test_request_larger_than_budget_fails_alone():
    reqs = reqs_of([dict(n=1 << 20, arrival_s=0.0), dict(n=1 << 30, arrival_s=0.001), dict(n=1 << 20, arrival_s=0.002)])
    st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=1 << 30, max_slots=2)
    assert [s["status"] for s in st] == [0, agg.E_NOMEM, 0]
    assert sm["failed"] == 1 and sm["completed"] == 2


def test_cache_hits_and_lru_eviction():
    # three distinct 1 GiB columns A, B, C, budget 2.5 GiB: A B A C A B
    n = (1 << 30) // 4
    seq = ["A", "B", "A", "C", "A", "B"]
    off = {"A": 0, "B": n, "C": 2 * n}
    cid = {"A": 1, "B": 2, "C": 3}
    reqs = reqs_of([dict(n=n, arrival_s=1.0 * i, offset=off[c], column_id=cid[c]) for i, c in enumerate(seq)])
    st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=(5 << 30) // 2, max_slots=2, cache_shipped=True)
    hits = [s["cache_hit"] for s in st]
    # A(miss) B(miss) A(hit) C(miss: evicts LRU = B) A(hit) B(miss: evicted)
    assert hits == [0, 0, 1, 0, 1, 0]
    assert sm["cache_hits"] == 2 and sm["bytes_shipped"] == 4 * n * 4
    st2, sm2 = agg.serve_simulate(reqs, hbm_budget_bytes=(5 << 30) // 2, max_slots=2, cache_shipped=False)
    assert sm2["cache_hits"] == 0 and sm2["bytes_shipped"] == 6 * n * 4


def test_latency_grows_with_load():
    lat = {}
    for rate in (50.0, 400.0):
        specs = request_stream(400, seed=2, n_min=10_000, n_max=1 << 28, rate_per_s=rate,
                               hot_items=1 << 28, arena_items=1 << 28)
        st, sm = agg.serve_simulate(reqs_of(specs), hbm_budget_bytes=8 << 30, max_slots=8, cache_shipped=False)
        lat[rate] = agg.percentile([s["done_s"] - s["arrival_s"] for s in st], 99)
    assert lat[400.0] > lat[50.0]


def test_invalid_requests_are_rejected():
    with pytest.raises(agg.AggError):   # arrivals out of order
        agg.serve_simulate(reqs_of([dict(n=10, arrival_s=1.0), dict(n=10, arrival_s=0.5)]), hbm_budget_bytes=1 << 20)
    with pytest.raises(agg.AggError):   # bad slot count
        agg.serve_simulate(reqs_of([dict(n=10, arrival_s=0.0)]), hbm_budget_bytes=1 << 20, max_slots=0)
    with pytest.raises(agg.AggError):   # bad op
        agg.serve_simulate([dict(ptr=4096, n=10, arrival_s=0.0, dtype="i32", op=9)], hbm_budget_bytes=1 << 20)


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert agg.percentile(xs, 50) == 50 and agg.percentile(xs, 99) == 99 and agg.percentile(xs, 100) == 100


def test_shipping_cap_keeps_resident_latency_low():
    specs = request_stream(600, seed=3, n_min=10_000, n_max=1 << 30, rate_per_s=150.0,
                           resident_frac=0.3, hot_items=1 << 30, arena_items=1 << 30)
    reqs = reqs_of(specs)
    out = {}
    for cap in (8, 2):
        st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=200 * 10**9, max_slots=8, cache_shipped=False,
                                    max_shipping=cap)
        res = [s["done_s"] - s["arrival_s"] for s, q in zip(st, specs) if q["resident"]]
        out[cap] = agg.percentile(res, 99)
        # never more shipped requests in flight than the cap
        ev = sorted([(s["admit_s"], 1) for s, q in zip(st, specs) if not q["resident"]] +
                    [(s["done_s"], -1) for s, q in zip(st, specs) if not q["resident"]], key=lambda e: (e[0], e[1]))
        live = peak = 0
        for _, d in ev:
            live += d
            peak = max(peak, live)
        assert peak <= cap
    assert out[2] < out[8]


def test_failed_shipped_request_is_not_cached():
    """A shipped request whose copy fails ends with AGG_E_HIP and leaves no
    cache entry: the next request for the same column ships it again (and
    that one, having succeeded, is then cached)."""
    n = 1 << 24
    reqs = reqs_of([dict(n=n, arrival_s=0.0, column_id=7), dict(n=n, arrival_s=1.0, column_id=7),
                    dict(n=n, arrival_s=2.0, column_id=7)])
    agg.fault_inject("ship", 1)
    try:
        st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=1 << 30, max_slots=2, cache_shipped=True)
    finally:
        agg.fault_inject("ship", 0)
    assert [s["status"] for s in st] == [agg.E_HIP, 0, 0]
    assert [s["cache_hit"] for s in st] == [0, 0, 1]
    assert [s["bytes_shipped"] for s in st] == [4 * n, 4 * n, 0]
    assert sm["failed"] == 1 and sm["completed"] == 2 and sm["cache_hits"] == 1
    # the failed request's region went back to the arena: a budget of one
    # column still serves the rest
    agg.fault_inject("ship", 1)
    try:
        st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=4 * n, max_slots=2, cache_shipped=True)
    finally:
        agg.fault_inject("ship", 0)
    assert [s["status"] for s in st] == [agg.E_HIP, 0, 0] and sm["peak_reserved_bytes"] <= 4 * n


def test_fault_countdown_and_disarm():
    reqs = reqs_of([dict(n=1 << 20, arrival_s=0.1 * i, column_id=i) for i in range(5)])
    agg.fault_inject("ship", 3)           # the third shipped copy fails
    try:
        st, _ = agg.serve_simulate(reqs, hbm_budget_bytes=1 << 30, max_slots=1, cache_shipped=False)
    finally:
        agg.fault_inject("ship", 0)
    assert [s["status"] for s in st] == [0, 0, agg.E_HIP, 0, 0]
    st, _ = agg.serve_simulate(reqs, hbm_budget_bytes=1 << 30, max_slots=1, cache_shipped=False)
    assert all(s["status"] == 0 for s in st)
    with pytest.raises(agg.AggError):
        agg.fault_inject(9, 1)
    with pytest.raises(agg.AggError):
        agg.fault_inject("ship", -1)


def test_fault_injection_from_the_environment():
    """AGG_FAULT_INJECT arms the countdowns at the library's first call (a
    fresh process, so the variable is read)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2606_10030_amd as agg\n"
        "reqs = [dict(ptr=1 << 20, n=1 << 20, arrival_s=0.1 * i, dtype='i32', op='sum', resident=False,"
        " column_id=i) for i in range(4)]\n"
        "st, sm = agg.serve_simulate(reqs, hbm_budget_bytes=1 << 30, max_slots=1, cache_shipped=False)\n"
        "print([s['status'] for s in st])\n" % root)
    env = dict(os.environ, AGG_FAULT_INJECT="alloc:5,ship:2")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == f"[0, {agg.E_HIP}, 0, 0]"
