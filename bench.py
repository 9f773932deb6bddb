"""Benchmark of the MI355X aggregation scan (one JSON line on stdout).

Workload: one column each of 2^30 int32, int64 and float32 items (uniform,
seeded), resident in HBM; one step runs SUM, MIN, MAX, COUNT and AVG on each
column through agg_run (float SUM / AVG in the default compensated mode).
`value` is the step's algorithmic bytes (every item read once per function that
reads items; COUNT reads none) divided by the step time.

Also reported, outside the timed steps: the per-cell GB/s and roofline
fraction, the dominant kernel's roofline (HIP events over the timed region),
the precision report (the three float modes on the precision-study column:
rel / abs_norm / kappa against the oracle's stored exact sum, and the a-priori
bound), the fused filter, the 2^20-item int32 SUM (per call, host enqueue and
GPU time), other readers of the same column for context (torch's sum, a device
copy), the Zipf and sorted columns, the paper's SF 50-200 sweep, group-by
over 2^28 rows, the end-to-end rate from pinned host memory (chunked copy
pipeline and zero-copy, raw and packed) with the measured host-to-device copy
ceiling, energy per aggregation, the 4096-column batch, serving (the scaled
configuration by default at 0.8 of the PCIe-bound load, with a sample checked
against the same requests run alone, and the same stream at loads 0.5 and 0.95),
and the CPU oracle's rate (cpu_baseline: the host's CPU share of
threads, one thread, and the host memory read ceiling).

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
PCIE_PEAK_GBS = 64.0           # PCIe Gen5 x16, one direction, nominal
METRIC = "aggregation GB/s and % of HBM peak (on-device + end-to-end), 1 MI355X"
N_ITEMS = 1 << 30
DTYPES = ["i32", "i64", "f32"]
OPS = ["sum", "min", "max", "count", "avg"]
WIDTH = {"i32": 4, "i64": 8, "f32": 4}
SEEDS = {"i32": 2, "i64": 3, "f32": 4}
KERNEL_SOURCES = ["paper_2606_10030_amd/csrc/agg_device.hpp", "paper_2606_10030_amd/csrc/agg_kernels.hip"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def settle(torch):
    """Hand cached device memory back and wait before a section that copies
    from the host: for about a second after device memory is freed,
    host-to-device copies run slower (most likely the driver clearing the
    freed memory with the same copy engines; measured: the 64 MiB-chunk copy
    pipeline at 31 instead of 56 GB/s right after a 4 GiB free, full speed
    1 s later; zero-copy reads are unaffected)."""
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    time.sleep(2.0)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, n_bytes_alg: int):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources and on a launch of the same
    algorithmic size; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if k is None or k.get("algorithmic_bytes") != n_bytes_alg:
        return None
    return k.get("hbm_bytes_per_launch")


def counters_mode(n: int):
    """Dispatches for hardware-counter runs: first 3 copies of 1 GiB (known
    traffic: 1 GiB read + 1 GiB written each), then 3 scans per dtype."""
    import torch
    import datagen
    import paper_2606_10030_amd as agg
    a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    o = torch.zeros(32, dtype=torch.uint8, device="cuda")
    for dt in DTYPES:
        tdt = {"i32": torch.int32, "i64": torch.int64, "f32": torch.float32}[dt]
        h = torch.empty(n, dtype=tdt, pin_memory=True)
        datagen.fill_ptr(h.data_ptr(), n, dt, "uniform", SEEDS[dt])
        d = h.to("cuda")
        p = agg.Plan(dt, "sum", max_n=n)
        for _ in range(3):
            p.enqueue(d, o)
        torch.cuda.synchronize()
        p.close()
        del d, h
    log("counters mode done")


def groupby_profile_mode(cards):
    """Dispatches for a kernel trace of group-by: 2^28 rows of int32 keys with
    each given number of distinct values, then 3 runs each of SUM(int64),
    SUM(float32) and COUNT; no JSON line."""
    import torch
    import datagen
    import paper_2606_10030_amd as agg
    n = 1 << 28
    dev = {}
    for dt in DTYPES:
        tdt = {"i32": torch.int32, "i64": torch.int64, "f32": torch.float32}[dt]
        h = torch.empty(n, dtype=tdt, pin_memory=True)
        datagen.fill_ptr(h.data_ptr(), n, dt, "uniform", SEEDS[dt])
        dev[dt] = h.to("cuda")
    for card in cards:
        keys = torch.remainder(dev["i32"].to(torch.int64) * 2654435761, card).to(torch.int32)
        for vdt, op in (("i64", "sum"), ("f32", "sum"), ("i32", "count")):
            g = agg.GroupBy("i32", vdt, op, max_n=n, max_groups=card)
            groups = torch.empty(card * agg.GROUP_BYTES, dtype=torch.uint8, device="cuda")
            ng = torch.zeros(1, dtype=torch.int64, device="cuda")
            for _ in range(3):
                g.enqueue(keys, dev[vdt], groups, ng)
            torch.cuda.synchronize()
            log(f"group-by {op}({vdt}) by {card} keys: {int(ng.item())} groups")
            g.close()
    log("group-by profile mode done")


POWER_MAX_W = 2800.0    # twice the MI355X board power: anything above is a misread
ENERGY_MIN_SPAN_S = 2.0  # the counter advances about once a second


def energy_power(edges, t_lo, t_hi, res_uj, max_w=POWER_MAX_W, min_span_s=ENERGY_MIN_SPAN_S):
    """Average power (W) from the GPU's cumulative energy counter.

    edges: [(time_s, counter)] at each observed change of the counter (one
    count = res_uj microjoules).  Only updates inside [t_lo, t_hi] count.
    Power comes from the intervals between consecutive updates: an interval
    whose counter goes backwards or implies more than max_w (a misread value,
    or a wrap) is dropped with its time, and the rest must span at least
    min_span_s seconds.  Returns (watts, info) or (None, info) with a reason."""
    inside = sorted((t, v) for t, v in edges if t_lo <= t <= t_hi)
    used_dt = used_j = 0.0
    used = rejected = 0
    for (ta, va), (tb, vb) in zip(inside, inside[1:]):
        dt = tb - ta
        dj = (vb - va) * res_uj * 1e-6
        if dt <= 0 or dj < 0 or dj > max_w * dt:
            rejected += 1
            continue
        used += 1
        used_dt += dt
        used_j += dj
    info = {"updates": len(inside), "intervals_used": used, "intervals_rejected": rejected,
            "span_s": round(used_dt, 3)}
    if len(inside) < 2:
        return None, {**info, "reason": "fewer than 2 counter updates inside the window"}
    if used_dt < min_span_s:
        return None, {**info, "reason": f"usable counter intervals span {used_dt:.3f} s < {min_span_s} s"}
    w = used_j / used_dt
    if not (0.0 < w <= max_w):
        return None, {**info, "reason": f"implausible average power {w:.4g} W"}
    return w, info


def batch_profile_mode(agg, torch, stream):
    """Dispatches for a kernel trace of the 4096-column batch (both
    configurations): 5 graph launches each after the autotuner; no JSON line."""
    out = bench_batch(agg, torch, stream, {"i32_sum": {"GB/s": None}}, separate=False)
    log(json.dumps(out))
    log("batch profile mode done")


def bench_energy(agg, torch, dev_i32, host_i32, stream):
    """Joules per aggregation from the GPU's energy accumulator (amdsmi), for
    the on-device SUM of a 2^30-item int32 column and the same SUM end to end
    (zero-copy from pinned host memory), plus idle power.

    The accumulator advances about once a second, so each figure comes from a
    window of several seconds: the host keeps the GPU busy with scans issued
    in batches and notes the time of every counter update; energy_power turns
    the updates inside the window into an average power (or None with the
    reason), and energy per scan = that power x the measured time per scan.
    The socket power reading, sampled through the same windows, is reported
    beside it as a cross-check."""
    try:
        import amdsmi
        amdsmi.amdsmi_init()
        h = amdsmi.amdsmi_get_processor_handles()[0]
        res = amdsmi.amdsmi_get_energy_count(h)["counter_resolution"]
    except Exception as ex:  # telemetry not available on this host
        return {"available": False, "reason": f"{type(ex).__name__}: {ex}"[:200]}

    def counter():
        return amdsmi.amdsmi_get_energy_count(h)["energy_accumulator"]

    def socket_w():
        try:
            pi = amdsmi.amdsmi_get_power_info(h)
        except Exception:
            return None
        for key in ("average_socket_power", "current_socket_power", "socket_power"):
            v = pi.get(key) if isinstance(pi, dict) else None
            if isinstance(v, (int, float)) and 0 < v <= POWER_MAX_W:
                return float(v)
        return None

    class Watch:
        def __init__(self):
            self.edges, self.last, self.sock, self.next_sock = [], counter(), [], 0.0

        def poll(self):
            now = time.perf_counter()
            v = counter()
            if v != self.last:
                self.edges.append((now, v))
                self.last = v
            if now >= self.next_sock:
                w = socket_w()
                if w is not None:
                    self.sock.append(w)
                self.next_sock = now + 0.02

        def socket_mean(self):
            return round(statistics.mean(self.sock), 1) if self.sock else None

    out = {"available": True, "source": "amdsmi energy accumulator (whole GPU), updates about once a second",
           "method": "energy_power: counter intervals inside a 6 s idle / 5 s busy window (misreads dropped, "
                     ">= 2 s of intervals, power in (0, 2800] W) x time per scan; socket power sampled "
                     "every 20 ms as a cross-check"}
    torch.cuda.synchronize()
    w = Watch()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 6.0:
        w.poll()
        time.sleep(0.001)
    idle_w, idle_info = energy_power(w.edges, t0, time.perf_counter(), res)
    out["idle_W"] = None if idle_w is None else round(idle_w, 1)
    out["idle"] = {**idle_info, "socket_power_W_mean": w.socket_mean()}
    n = dev_i32.numel()
    o = torch.zeros(32, dtype=torch.uint8, device="cuda")
    for label, src, col, batch in (("on_device", "device", dev_i32, 200), ("end_to_end_zerocopy", "zerocopy", host_i32, 2)):
        p = agg.Plan("i32", "sum", max_n=n, src=src)
        p.enqueue(col, o, stream=stream)
        torch.cuda.synchronize()
        w, pending, scans = Watch(), [], 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 5.0 or pending:
            if time.perf_counter() - t0 < 5.0 and len(pending) < 3:
                for _ in range(batch):
                    p.enqueue(col, o, stream=stream)
                ev = torch.cuda.Event()
                ev.record(stream)
                pending.append(ev)
                scans += batch
            else:
                w.poll()
                if pending and pending[0].query():
                    pending.pop(0)
                else:
                    time.sleep(0.0005)
        t1 = time.perf_counter()
        p.close()
        per_scan_s = (t1 - t0) / scans
        busy_w, busy_info = energy_power(w.edges, t0, t1, res)
        gb = n * 4 / 1e9
        rec = {"scans": scans, "seconds": round(t1 - t0, 2), "ms_per_scan": round(per_scan_s * 1e3, 3),
               "counter": busy_info, "socket_power_W_mean": w.socket_mean()}
        if busy_w is None:
            out[label] = {**rec, "J_per_scan": None}
            continue
        per = busy_w * per_scan_s
        out[label] = {**rec, "J_per_scan": round(per, 4),
                      "J_per_scan_above_idle": None if idle_w is None else round((busy_w - idle_w) * per_scan_s, 4),
                      "J_per_GB": round(per / gb, 4), "avg_W": round(busy_w, 1),
                      "J_for_1.2e9_items": round(per * 1.2e9 / n, 4)}
    try:
        amdsmi.amdsmi_shut_down()
    except Exception:
        pass
    return out


def bench_batch(agg, torch, stream, table, separate=True):
    """4096 columns, lengths log-uniform in [1e3, 1e7], dtype uniform over int32 /
    int64 / float32, function uniform over SUM / MIN / MAX / AVG (seed 12); also
    the same columns rescaled to 2^30 items in total."""
    import numpy as np
    import datagen
    r = np.random.default_rng(12)
    ncols = 4096
    lens = np.floor(np.exp(r.uniform(np.log(1e3), np.log(1e7), ncols))).astype(np.int64)
    dts = [DTYPES[i] for i in r.integers(0, 3, ncols)]
    ops = [["sum", "min", "max", "avg"][i] for i in r.integers(0, 4, ncols)]
    out = {}
    for label, scale in (("log_uniform_1e3_1e7", 1.0), ("rescaled_to_2^30_items", None)):
        ln = lens if scale else np.maximum(1, np.floor(lens * (N_ITEMS / lens.sum()))).astype(np.int64)
        tdt = {"i32": torch.int32, "i64": torch.int64, "f32": torch.float32}
        # one device buffer per dtype, columns at 256-byte aligned offsets
        offs, tot = [], {d: 0 for d in DTYPES}
        for dt, n in zip(dts, ln):
            offs.append(tot[dt])
            tot[dt] += -(-int(n) * WIDTH[dt] // 256) * 256 // WIDTH[dt]
        bufs = {d: torch.empty(max(1, tot[d]), dtype=tdt[d], device="cuda") for d in DTYPES}
        stage = torch.empty(int(ln.max()) * 8, dtype=torch.uint8, pin_memory=True)
        t0 = time.time()
        for i, (dt, n) in enumerate(zip(dts, ln)):
            datagen.fill_ptr(stage.data_ptr(), int(n), dt, "uniform", 1000 + i)
            dst = bufs[dt][offs[i]:offs[i] + int(n)]
            dst.view(torch.uint8).copy_(stage[:int(n) * WIDTH[dt]], non_blocking=False)
        log(f"batch columns ({label}) generated in {time.time() - t0:.1f}s")
        cols = [agg.BatchColumn(bufs[dt][offs[i]:offs[i] + int(n)], ops[i]) for i, (dt, n) in enumerate(zip(dts, ln))]
        total_bytes = int(sum(int(n) * WIDTH[dt] for dt, n in zip(dts, ln)))
        b = agg.Batch(cols)
        tuned, tuned_ms = b.autotune(stream)
        res = torch.zeros(ncols * 32, dtype=torch.uint8, device="cuda")
        for _ in range(2):
            b.enqueue(res, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            b.enqueue(res, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        gbs = total_bytes / (ms * 1e-3) / 1e9
        rec = {"columns": ncols, "items": int(ln.sum()), "bytes": total_bytes, "graph_ms": round(ms, 3),
               "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
               "tuned": {"unroll": tuned.unroll, "waves_per_block": tuned.waves_per_block,
                         "blocks_per_cu": tuned.blocks_per_cu},
               "work_items": b.info()["nitems"],
               "plain_single_column_i32_sum_GB/s": table["i32_sum"]["GB/s"]}
        out[label] = rec
        if not separate:
            b.close()
            del bufs, cols, stage
            torch.cuda.empty_cache()
            continue
        # the same columns as 4096 separate agg_run calls
        plans = {}
        for c, dt in zip(cols, dts):
            key = (dt, c.op)
            if key not in plans:
                plans[key] = agg.Plan(dt, c.op, max_n=int(ln.max()))
        o = torch.zeros(32, dtype=torch.uint8, device="cuda")
        for c, dt in zip(cols, dts):
            plans[(dt, c.op)].enqueue(c.col, o, stream=stream)
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        for c, dt in zip(cols, dts):
            plans[(dt, c.op)].enqueue(c.col, o, stream=stream)
        e3.record(stream)
        torch.cuda.synchronize()
        ms_sep = e2.elapsed_time(e3)
        rec["separate_agg_run_ms"] = round(ms_sep, 3)
        rec["separate_GB/s"] = round(total_bytes / (ms_sep * 1e-3) / 1e9, 1)
        for p in plans.values():
            p.close()
        b.close()
        del bufs, cols, stage
        torch.cuda.empty_cache()
    return out


def bench_groupby(agg, torch, stream, dev):
    """Group-by over 2^28 rows: int32 keys of a given number of distinct values
    (a multiplicative hash of the uniform int32 column, reduced mod the
    cardinality) with int64 or float32 values.  Bytes = keys + values read once."""
    n = 1 << 28
    out = {}
    for card in (16, 1024, 8192, 1 << 16, 1 << 20):
        keys = torch.remainder(dev["i32"][:n].to(torch.int64) * 2654435761, card).to(torch.int32)
        for vdt, op in (("i64", "sum"), ("f32", "sum"), ("i32", "count")):
            g = agg.GroupBy("i32", vdt, op, max_n=n, max_groups=card)
            groups = torch.empty(card * agg.GROUP_BYTES, dtype=torch.uint8, device="cuda")
            ng = torch.zeros(1, dtype=torch.int64, device="cuda")
            vals = dev[vdt][:n]
            for _ in range(2):
                g.enqueue(keys, vals, groups, ng, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(5):
                g.enqueue(keys, vals, groups, ng, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            b = n * (4 + (0 if op == "count" else WIDTH[vdt]))
            out[f"{op}_{vdt}_by_i32_card{card}"] = {
                "ms": round(ms, 4), "GB/s": round(b / (ms * 1e-3) / 1e9, 1),
                "Grows/s": round(n / (ms * 1e-3) / 1e9, 2), "hbm_frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "groups": int(ng.item())}
            g.close()
        del keys
    return out


def bench_serve(agg, torch, host_i32, dev_i32, full=False, rho=0.8):
    """Poisson stream of int32 requests, lengths log-uniform in [1e4, n_max],
    30% resident (slices of a column in HBM) and 70% shipped from pinned host
    memory, admitted by a 200 GB HBM budget, at rho of the PCIe-bound capacity."""
    from datagen.serving import mean_bytes, request_stream
    nreq, n_max = (10_000, 1 << 33) if full else (1000, 1 << 30)
    arena_h = host_i32
    if full:
        arena_h = torch.empty(n_max, dtype=torch.int32, pin_memory=True)
        import datagen
        datagen.fill_ptr(arena_h.data_ptr(), n_max, "i32", "uniform", 13)
        log(f"serving arena: {n_max} int32 items in pinned host memory")
    cap = 55e9 / (0.7 * mean_bytes(10_000, n_max, 4))
    rate = rho * cap
    specs = request_stream(nreq, seed=13, n_min=10_000, n_max=n_max, rate_per_s=rate, resident_frac=0.3,
                           hot_items=dev_i32.numel(), arena_items=arena_h.numel())
    reqs = [dict(ptr=(dev_i32 if s["resident"] else arena_h).data_ptr() + 4 * s["offset"], n=s["n"],
                 column_id=s["column_id"], arrival_s=s["arrival_s"], dtype="i32", op=s["op"],
                 resident=s["resident"]) for s in specs]
    budget = 200 * 10**9
    free, _ = torch.cuda.mem_get_info()
    budget = min(budget, int(free - (8 << 30)))
    srv = agg.Server(hbm_budget_bytes=budget, max_slots=8, cache_shipped=False, max_shipping=2,
                     progress_every=1000 if full else 0)
    log(f"serving {nreq} requests (lengths up to {n_max}) at {rate:.1f}/s")
    t0 = time.time()
    results, stats, sm = srv.run(reqs)
    wall = time.time() - t0
    srv.close()
    # a seeded sample of the results, each against the same request run alone
    # (agg_run on the same canonical shape: the bits must be identical)
    import numpy as np
    sample = sorted(np.random.default_rng(14).choice(len(reqs), size=min(64, len(reqs)), replace=False).tolist())
    mism = 0
    o = torch.zeros(32, dtype=torch.uint8, device="cuda")
    for i in sample:
        q = reqs[i]
        p = agg.Plan("i32", q["op"], max_n=q["n"], src="device" if q["resident"] else "zerocopy")
        p.enqueue(q["ptr"], o, n=q["n"])
        torch.cuda.synchronize()
        alone = agg.parse_results(o.cpu().numpy().tobytes(), [(agg.I32, agg.OPS[q["op"]])])[0]
        p.close()
        got = results[i]
        if (got["i64"], got["f64"], got["count"], got["is_null"]) != \
                (alone["i64"], alone["f64"], alone["count"], alone["is_null"]) or stats[i]["status"] != 0:
            mism += 1
    lat = [s["done_s"] - s["arrival_s"] for s in stats]
    lat_res = [s["done_s"] - s["arrival_s"] for s, q in zip(stats, reqs) if q["resident"]]
    lat_ship = [s["done_s"] - s["arrival_s"] for s, q in zip(stats, reqs) if not q["resident"]]
    return {"configuration": "full" if full else
            "scaled: 10^3 requests up to 2^30 items (the full 10^4 requests up to 2^33 run with --serve-full "
            "and in tests/test_gpu_serve.py with AGG_SERVE_FULL=1)",
            "checked_vs_alone": len(sample), "mismatches_vs_alone": mism,
            "requests": nreq, "n_range": [10_000, n_max], "load_rho": rho, "arrival_rate_per_s": round(rate, 1),
            "hbm_budget_bytes": budget, "max_slots": 8, "max_shipping": 2,
            "completed": sm["completed"], "failed": sm["failed"],
            "p50_ms": round(agg.percentile(lat, 50) * 1e3, 3), "p99_ms": round(agg.percentile(lat, 99) * 1e3, 3),
            "resident_p50_ms": round(agg.percentile(lat_res, 50) * 1e3, 3),
            "resident_p99_ms": round(agg.percentile(lat_res, 99) * 1e3, 3),
            "shipped_p50_ms": round(agg.percentile(lat_ship, 50) * 1e3, 3),
            "shipped_p99_ms": round(agg.percentile(lat_ship, 99) * 1e3, 3),
            "makespan_s": round(sm["makespan_s"], 3), "wall_s": round(wall, 3),
            "scanned_GB/s": round(sm["bytes_scanned"] / sm["makespan_s"] / 1e9, 2),
            "shipped_GB/s": round(sm["bytes_shipped"] / sm["makespan_s"] / 1e9, 2),
            "bytes_scanned": sm["bytes_scanned"], "bytes_shipped": sm["bytes_shipped"],
            "peak_busy_slots": sm["peak_busy_slots"], "peak_reserved_bytes": sm["peak_reserved_bytes"]}


def bench_precision(agg, torch, stream, dev_f32):
    """Float32 SUM in the three precision modes on the precision-study column
    (2^30 items, N(0,1) with 1% of +-1e6, seed 11) and on the benchmark's
    uniform float32 column (seed 4): time per launch, and the error against
    the exact sum stored by tests/golden/make_precision_refs.py (the oracle's
    value, computed ahead of time): rel, abs_norm, kappa, and the library's
    a-priori bound."""
    import datagen
    refs = json.load(open(os.path.join(ROOT, "tests", "golden", "precision_refs.json")))["columns"]
    n = N_ITEMS
    h = torch.empty(n, dtype=torch.float32, pin_memory=True)
    datagen.fill_ptr(h.data_ptr(), n, "f32", "normal_outliers", 11)
    d_c3 = h.to("cuda")
    del h
    out = {}
    for name, col in (("f32_normal_outliers_seed11", d_c3), ("f32_uniform_seed4", dev_f32)):
        ref = refs[name]
        if col.numel() != ref["n"]:
            continue
        exact, a = ref["exact_sum"], ref["abs_sum"]
        modes = {}
        for prec in ("f32", "f64_combine", "neumaier"):
            p = agg.Plan("f32", "sum", max_n=n, prec=prec)
            o = torch.zeros(32, dtype=torch.uint8, device="cuda")
            for _ in range(2):
                p.enqueue(col, o, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(5):
                p.enqueue(col, o, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            got = agg.parse_results(o.cpu().numpy().tobytes(), [(agg.F32, agg.SUM)])[0]["f64"]
            p.close()
            err = abs(got - exact)
            bound = agg.float_sum_bound_coeff(prec, n) * a
            modes[prec] = {"value": got, "rel": err / abs(exact), "abs_norm": err / a,
                           "apriori_rel_bound": bound / abs(exact), "within_bound": err <= bound,
                           "ms": round(ms, 4), "GB/s": round(n * 4 / (ms * 1e-3) / 1e9, 1)}
        out[name] = {"n": n, "exact_sum": exact, "kappa": a / abs(exact), "modes": modes}
    del d_c3
    return out


def bench_distributions(agg, torch, stream, plans, hbuf, dbuf):
    """The other distributions of the 2^30-item columns (Zipf(1.1) on ranks
    [1, 2^20], and the uniform column sorted ascending): SUM / MIN / MAX / AVG
    per dtype, 3 launches each (the seeds of the full-size GPU tests)."""
    import datagen
    n = N_ITEMS
    out = {}
    for dt in DTYPES:
        for dist, ds in (("zipf", 1), ("sorted", 2)):
            seed = {"i32": 2, "i64": 5, "f32": 8}[dt] + ds
            t0 = time.time()
            datagen.fill_ptr(hbuf.data_ptr(), n, dt, dist, seed)
            nb = n * WIDTH[dt]
            dbuf[:nb].copy_(hbuf[:nb])
            col = dbuf[:nb].view({"i32": torch.int32, "i64": torch.int64, "f32": torch.float32}[dt])
            log(f"distribution {dt} {dist}: generated + copied in {time.time() - t0:.1f}s")
            for op in ("sum", "min", "max", "avg"):
                o = torch.zeros(32, dtype=torch.uint8, device="cuda")
                plans[(dt, op)].enqueue(col, o, stream=stream)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(3):
                    plans[(dt, op)].enqueue(col, o, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / 3
                gbs = nb / (ms * 1e-3) / 1e9
                out[f"{dt}_{dist}_{op}"] = {"ms": round(ms, 4), "GB/s": round(gbs, 1),
                                            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def bench_sf_sweep(agg, torch, stream, hbuf, dbuf):
    """The paper's scalability sweep (Section 5.2): SUM over an int32 key column
    uniform in [1, 1e4 * SF] with 6e6 * SF rows, SF 50 / 100 / 150 / 200, on
    device (5 launches) and end to end by zero-copy from pinned host memory."""
    import datagen
    out = {}
    for sf in (50, 100, 150, 200):
        n = 6_000_000 * sf
        datagen.fill_ptr(hbuf.data_ptr(), n, "i32", "uniform", 31, 1, 10_000 * sf + 1)
        dbuf[:n * 4].copy_(hbuf[:n * 4])
        rec = {"rows": n, "bytes": n * 4}
        for src, col, reps in (("device", dbuf[:n * 4].view(torch.int32), 5),
                               ("zerocopy", hbuf[:n * 4].view(torch.int32), 2)):
            p = agg.Plan("i32", "sum", max_n=n, src=src)
            o = torch.zeros(32, dtype=torch.uint8, device="cuda")
            p.enqueue(col, o, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                p.enqueue(col, o, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            p.close()
            rec[src] = {"ms": round(ms, 4), "rows/s": round(n / (ms * 1e-3), 1),
                        "GB/s": round(n * 4 / (ms * 1e-3) / 1e9, 1)}
        out[f"SF{sf}"] = rec
    return out


def bench_device_reference(torch, dev):
    """Other readers of the same 2^30-item columns on the same device, for
    context beside the scan's rate: torch's own sums (read-only reductions;
    int32 with int64 accumulation, float32) and a device-to-device copy of
    the int32 column (counted as read + written bytes)."""
    x = dev["i32"]
    nbytes = x.numel() * 4

    def timed(f, reps=5):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_sum = timed(lambda: torch.sum(x, dtype=torch.int64))
    ms_fsum = timed(lambda: torch.sum(dev["f32"]))
    y = torch.empty_like(x)
    ms_copy = timed(lambda: y.copy_(x))
    del y
    return {"torch_sum_i32_GB/s": round(nbytes / (ms_sum * 1e-3) / 1e9, 1),
            "torch_sum_f32_GB/s": round(nbytes / (ms_fsum * 1e-3) / 1e9, 1),
            "d2d_copy_read_plus_write_GB/s": round(2 * nbytes / (ms_copy * 1e-3) / 1e9, 1),
            "note": "same device and column, other kernels: context for the scan's fraction of the 8 TB/s peak"}


def bench_small_call(agg, torch, stream, dev_i32):
    """The 2^20-item int32 SUM (launch-bound): time per call back to back on
    one stream, the host's enqueue time per call (Python binding + library),
    the GPU's own time per call, measured with the calls queued behind
    enough earlier work that the host is never the limit, and the latency of
    one call (enqueue, then wait for the stream) with nothing else queued."""
    small = dev_i32[: 1 << 20]
    p = agg.Plan("i32", "sum", max_n=1 << 20)
    o = torch.zeros(32, dtype=torch.uint8, device="cuda")
    for _ in range(50):
        p.enqueue(small, o, stream=stream)
    torch.cuda.synchronize()
    calls = 1000
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(calls):
        p.enqueue(small, o, stream=stream)
    e1.record(stream)
    host_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    back_to_back_us = e0.elapsed_time(e1) / calls * 1e3
    # queue the calls behind ~30 ms of scans so every call is enqueued before the first runs
    pb = agg.Plan("i32", "sum", max_n=dev_i32.numel())
    ob = torch.zeros(32, dtype=torch.uint8, device="cuda")
    for _ in range(50):
        pb.enqueue(dev_i32, ob, stream=stream)
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record(stream)
    for _ in range(calls):
        p.enqueue(small, o, stream=stream)
    e3.record(stream)
    torch.cuda.synchronize()
    gpu_us = e2.elapsed_time(e3) / calls * 1e3
    lat = []
    for _ in range(300):
        t1 = time.perf_counter()
        p.enqueue(small, o, stream=stream)
        stream.synchronize()
        lat.append((time.perf_counter() - t1) * 1e6)
    lat.sort()
    pb.close()
    p.close()
    return {"us_per_call_back_to_back": round(back_to_back_us, 2),
            "host_enqueue_us_per_call": round(host_s / calls * 1e6, 2),
            "gpu_us_per_call_queued": round(gpu_us, 2),
            "latency_us_p50": round(lat[len(lat) // 2], 2),
            "latency_us_p99": round(lat[int(len(lat) * 0.99)], 2),
            "launches_per_call": 1,
            "note": "one launch per call at this size (the scan's last workgroup merges the 256 partials); "
                    "gpu_us_per_call_queued: events around calls queued behind ~30 ms of earlier scans; "
                    "latency: enqueue then stream synchronize, 300 calls"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(host, cells, step_bytes, n):
    """The oracle (plain, exact, untuned) over the step's cells on the host:
    whole steps for about 10 s with the host's CPU share of threads, a
    1-thread run over one 2^28-item column, and the host memory read ceiling
    (a multi-threaded read of the three host columns)."""
    import oracle
    threads = oracle.default_threads()     # OMP_NUM_THREADS: the CPU share of this GPU's job
    cells_cpu = [c for c in cells if c[1] != "count"]
    code = {"i32": 0, "i64": 1, "f32": 2}
    opc = {"sum": 0, "min": 1, "max": 2, "avg": 4}
    t0 = time.perf_counter()
    reps = 0
    while reps == 0 or time.perf_counter() - t0 < 10.0:   # whole steps, about 10 s of CPU work
        for dt, op in cells_cpu:
            oracle.aggregate_ptr(host[dt].data_ptr(), n, code[dt], opc[op], threads)
        reps += 1
    cpu_s = time.perf_counter() - t0
    m1 = min(n, 1 << 28)
    t1 = time.perf_counter()
    oracle.aggregate_ptr(host["i32"].data_ptr(), m1, 0, 0, 1)
    one_s = time.perf_counter() - t1
    ceil = {}
    for th in sorted({1, threads}):
        t2 = time.perf_counter()
        nbytes = 0
        for dt in DTYPES:
            oracle.read_ceiling(host[dt].data_ptr(), n * WIDTH[dt], th)
            nbytes += n * WIDTH[dt]
        ceil[th] = round(nbytes / (time.perf_counter() - t2) / 1e9, 2)
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": round(reps * step_bytes / cpu_s / 1e9, 2), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} full step(s): {len(cells_cpu)} cells each over the same 2^30-item columns "
                      f"({step_bytes / 2**30:.0f} GiB read per step), {cpu_s:.1f} s",
            "threads": threads, "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
            "affinity_cpus": affinity,
            "threads_note": "threads = OMP_NUM_THREADS, the host CPU share given to one GPU's job",
            "one_thread_GB/s": round(m1 * 4 / one_s / 1e9, 2),
            "one_thread_sample": f"int32 SUM over {m1} items",
            "host_read_ceiling_GB/s": ceil[threads], "host_read_ceiling_1_thread_GB/s": ceil[1]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-e2e", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--no-groupby", action="store_true")
    ap.add_argument("--no-dists", action="store_true", help="skip the Zipf / sorted cells and the SF sweep")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving with 10^4 requests of up to 2^33 int32 items (minutes of PCIe time)")
    ap.add_argument("--n", type=int, default=N_ITEMS, help=argparse.SUPPRESS)
    ap.add_argument("--counters", action="store_true",
                    help="profiling mode for rocprofv3 --pmc: a 1 GiB device copy (calibration) "
                         "then 3 launches of each int32/int64/float32 SUM scan; no JSON line")
    ap.add_argument("--profile-batch", action="store_true",
                    help="profiling mode for a rocprofv3 kernel trace of the 4096-column batch; no JSON line")
    ap.add_argument("--profile-groupby", type=int, nargs="+", metavar="GROUPS",
                    help="profiling mode for a rocprofv3 kernel trace: group-by over 2^28 rows with "
                         "the given key counts; no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the scan's only cross-GPU step would be a 32-byte partial exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    import paper_2606_10030_amd as agg

    torch.cuda.set_device(0)
    info = agg.device_info(0)
    n = args.n
    stream = torch.cuda.current_stream()

    if args.counters:
        counters_mode(n)
        return
    if args.profile_groupby:
        groupby_profile_mode(args.profile_groupby)
        return
    if args.profile_batch:
        batch_profile_mode(agg, torch, stream)
        return

    # ---- inputs: generated into pinned host memory, copied to HBM
    host, dev = {}, {}
    for dt in DTYPES:
        t0 = time.time()
        tdt = {"i32": torch.int32, "i64": torch.int64, "f32": torch.float32}[dt]
        h = torch.empty(n, dtype=tdt, pin_memory=True)
        datagen.fill_ptr(h.data_ptr(), n, dt, "uniform", SEEDS[dt])
        host[dt] = h
        dev[dt] = h.to("cuda", non_blocking=False)
        log(f"input {dt}: {n} items generated and copied in {time.time() - t0:.1f}s")
    torch.cuda.synchronize()

    plans = {(dt, op): agg.Plan(dt, op, max_n=n) for dt in DTYPES for op in OPS}
    outs = torch.zeros(len(plans) * 32, dtype=torch.uint8, device="cuda")
    cells = list(plans.keys())

    # The dominant kernel is the one that reads the most bytes per step: the int64
    # SUM scan, which the SUM and AVG cells share (two 8 GiB launches per step).
    # Only its launches are bracketed by HIP events inside the timed steps: an
    # event pair leaves about 10 us of idle queue time behind it, which would
    # otherwise be charged to every cell of the step.
    dom = "i64_sum"
    dom_idx = [i for i, (dt, op) in enumerate(cells) if dt == "i64" and op in ("sum", "avg")]

    def step(ev=None):
        for i, (dt, op) in enumerate(cells):
            timed = ev is not None and i in dom_idx
            if timed:
                ev[dom_idx.index(i)][0].record(stream)
            plans[(dt, op)].enqueue(dev[dt], outs[i * 32:(i + 1) * 32], stream=stream)
            if timed:
                ev[dom_idx.index(i)][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in dom_idx]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    bytes_of = {c: (0 if c[1] == "count" else n * WIDTH[c[0]]) for c in cells}
    step_bytes = sum(bytes_of.values())
    ms_per_step = wall * 1e3 / args.steps
    value = step_bytes / (ms_per_step * 1e-3) / 1e9

    dom_times = [ev[s][j][0].elapsed_time(ev[s][j][1]) for s in range(args.steps) for j in range(len(dom_idx))]
    dom_ms = statistics.mean(dom_times)
    dom_bytes = n * WIDTH["i64"]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom, dom_bytes),
                "kernel": f"scan {dom}: HIP events in the timed steps bracket each int64 SUM / AVG agg_run "
                          "call (scan launch + one-workgroup combine launch), on the stream both are launched on",
                "algorithmic_bytes_per_launch": dom_bytes, "avg_launch_ms": round(dom_ms, 4),
                "launches_timed": len(dom_times)}

    # ---- per-cell rates (after the timed steps: 3 back-to-back launches per cell between events)
    table = {}
    for i, c in enumerate(cells):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            plans[c].enqueue(dev[c[0]], outs[i * 32:(i + 1) * 32], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        m = e0.elapsed_time(e1) / 3
        gbs = bytes_of[c] / (m * 1e-3) / 1e9 if bytes_of[c] else None
        table[f"{c[0]}_{c[1]}"] = {"ms": round(m, 4), "GB/s": None if gbs is None else round(gbs, 1),
                                   "rows/s": round(n / (m * 1e-3), 1),
                                   "hbm_frac": None if gbs is None else round(gbs / HBM_PEAK_GBS, 4)}

    extra = {}
    # ---- float precision: the three modes on the precision-study column and on the step's float32 column
    extra["precision"] = bench_precision(agg, torch, stream, dev["f32"])

    # ---- fused filter + aggregate: SUM(x) WHERE y < 0 (half the items), both columns read once
    fused = {}
    for vdt, fdt in (("i32", "f32"), ("i64", "i32"), ("f32", "i32")):
        p = agg.Plan(vdt, "sum", max_n=n)
        filt = agg.make_filter(dev[fdt], None, 0, True, False)
        o = torch.zeros(32, dtype=torch.uint8, device="cuda")
        for _ in range(2):
            p.enqueue_filtered(dev[vdt], filt, o, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            p.enqueue_filtered(dev[vdt], filt, o, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        b = n * (WIDTH[vdt] + WIDTH[fdt])
        fused[f"sum_{vdt}_where_{fdt}_lt_0"] = {"ms": round(ms, 4), "GB/s": round(b / (ms * 1e-3) / 1e9, 1),
                                                "hbm_frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        p.close()
    extra["fused_filter"] = fused

    # ---- latency: 2^20 int32 SUM (launch-bound)
    c1 = bench_small_call(agg, torch, stream, dev["i32"])
    extra["i32_sum_2e20_us_per_call"] = c1["us_per_call_back_to_back"]
    extra["i32_sum_2e20"] = c1
    extra["device_reference"] = bench_device_reference(torch, dev)

    # ---- the other distributions and the paper's SF sweep (one spare 8 GiB buffer on each side)
    if not args.no_dists:
        hbuf = torch.empty(n * 8, dtype=torch.uint8, pin_memory=True)
        dbuf = torch.empty(n * 8, dtype=torch.uint8, device="cuda")
        extra["distributions"] = bench_distributions(agg, torch, stream, plans, hbuf, dbuf)
        extra["sf_sweep"] = bench_sf_sweep(agg, torch, stream, hbuf, dbuf)
        del hbuf, dbuf
        torch.cuda.empty_cache()

    # ---- group-by aggregation (per-key SUM / COUNT over 2^28 rows)
    if not args.no_groupby:
        extra["groupby"] = bench_groupby(agg, torch, stream, dev)

    # ---- end to end from pinned host memory
    if not args.no_e2e:
        settle(torch)
        e2e = {}
        # every plan (and its staging ring) is made first, and the copy engines
        # are left a moment to finish clearing new device memory, so that no
        # timed copy shares them with the driver's clearing
        plans = {(src, dt): agg.Plan(dt, "sum", max_n=n, src=src)
                 for src in ("pinned_host", "zerocopy") for dt in DTYPES}
        dst = torch.empty_like(dev["i32"])
        torch.cuda.synchronize()
        time.sleep(2.0)
        for src in ("pinned_host", "zerocopy"):
            for dt in DTYPES:
                p = plans[(src, dt)]
                # one untimed full run first: after the link has idled, the first 100 ms or so
                # of host-to-device traffic run slower (measured: 48.5 GB/s for the first staged
                # scan in a process, 55.9 GB/s for the same scan repeated)
                p.enqueue(host[dt], o, stream=stream)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0 = time.perf_counter()
                e0.record(stream)
                p.enqueue(host[dt], o, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                wall_s = time.perf_counter() - t0
                gbs = n * WIDTH[dt] / (e0.elapsed_time(e1) * 1e-3) / 1e9
                e2e[f"{src}_{dt}_sum"] = {"GB/s": round(gbs, 2), "pcie_frac": round(gbs / PCIE_PEAK_GBS, 3),
                                          "wall_ms": round(wall_s * 1e3, 2)}
        # the host-to-device ceiling: one plain copy of the int32 column
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dst.copy_(host["i32"], non_blocking=True)
        e1.record(stream)
        torch.cuda.synchronize()
        h2d = n * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        e2e["h2d_copy_GB/s"] = round(h2d, 2)
        for k, v in e2e.items():
            if isinstance(v, dict) and "GB/s" in v:
                v["h2d_ceiling_frac"] = round(v["GB/s"] / h2d, 3)
        del dst
        for p in plans.values():
            p.close()
        # frame-of-reference + bit-packed int32 (compression cuts the PCIe bytes)
        t0 = time.perf_counter()
        pc = agg.pack_i32(host["i32"].numpy())
        pack_s = time.perf_counter() - t0
        for src, where in (("zerocopy", "pinned"), ("device", "cuda")):
            col = pc.to(where)
            p = agg.Plan("i32", "sum", max_n=n, src=src)
            p.enqueue_packed(col, o, stream=stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 2 if src == "zerocopy" else 5
            e0.record(stream)
            for _ in range(reps):
                p.enqueue_packed(col, o, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            e2e[f"packed_{src}_i32_sum"] = {"raw_equivalent_GB/s": round(n * 4 / (ms * 1e-3) / 1e9, 2),
                                            "packed_GB/s": round(pc.nbytes / (ms * 1e-3) / 1e9, 2),
                                            "ms": round(ms, 3)}
            p.close()
            del col
        e2e["packed_ratio"] = round(pc.nbytes / (n * 4), 4)
        e2e["pack_host_s"] = round(pack_s, 3)
        e2e["packed_zerocopy_speedup_vs_raw_zerocopy"] = round(
            e2e["packed_zerocopy_i32_sum"]["raw_equivalent_GB/s"] / e2e["zerocopy_i32_sum"]["GB/s"], 3)
        del pc
        dev_ms = table["i32_sum"]["ms"]
        e2e_ms = n * 4 / (e2e["pinned_host_i32_sum"]["GB/s"] * 1e9) * 1e3
        e2e["transfer_share_of_e2e_time"] = round(1 - dev_ms / e2e_ms, 4)
        extra["e2e"] = e2e

    # ---- energy per aggregation (on-device and end to end)
    if not args.no_energy:
        extra["energy"] = bench_energy(agg, torch, dev["i32"], host["i32"], stream)

    # ---- batch: 4096 mixed columns in one persistent launch under a HIP graph
    if not args.no_batch:
        extra["batch"] = bench_batch(agg, torch, stream, table)

    # ---- serving: Poisson requests, 30% resident / 70% shipped, HBM budget
    if not args.no_serve:
        settle(torch)
        extra["serve"] = bench_serve(agg, torch, host["i32"], dev["i32"], full=args.serve_full)
        # the same scaled stream at the two other loads of the serving configuration
        keep = ("load_rho", "arrival_rate_per_s", "completed", "failed", "mismatches_vs_alone", "p50_ms", "p99_ms",
                "resident_p50_ms", "resident_p99_ms", "shipped_p50_ms", "shipped_p99_ms", "makespan_s",
                "shipped_GB/s")
        extra["serve_load_sweep"] = {
            f"rho_{r}": {k: v for k, v in bench_serve(agg, torch, host["i32"], dev["i32"], rho=r).items() if k in keep}
            for r in (0.5, 0.95)}

    # ---- CPU oracle baseline (rank 0, N = 1): one step's cells on the host cores
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(host, cells, step_bytes, n)

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64,f32",
        "data": "synthetic",
        "config": {"workload": "aggregation scan of 2^30-item int32, int64 and float32 columns "
                               "(uniform), SUM/MIN/MAX/COUNT/AVG, resident in HBM",
                   "n": n, "bytes_per_step": step_bytes, "parallelism": "single GPU",
                   "device": info},
        "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "rows_per_s": round(n * sum(1 for c in cells if c[1] != "count") / (ms_per_step * 1e-3), 1),
        "rows_per_s_note": "rows read per second: the 12 cells that read the column (COUNT reads nothing)",
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cells": table,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
