"""bench.py's output contract: one JSON line with the required fields, a
roofline object consistent with itself, and a refusal of more than one GPU."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", BENCH)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)   # top level imports only the standard library
    return mod


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_profiled_kernel_and_size():
    bench = load_bench()
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as f:
        stored = json.load(f)
    k = stored["kernels"]["i64_sum"]
    got = bench.traffic_for("i64_sum", k["algorithmic_bytes"])
    if stored["kernel_source_hash"] == bench.kernel_source_hash():
        assert got == k["hbm_bytes_per_launch"]
    else:
        assert got is None                      # counters taken on other kernel sources
    assert bench.traffic_for("i64_sum", k["algorithmic_bytes"] // 2) is None
    assert bench.traffic_for("no_such_kernel", k["algorithmic_bytes"]) is None


@pytest.mark.gpu
def test_bench_prints_one_contract_line():
    r = subprocess.run([sys.executable, "-u", BENCH, "--steps", "2", "--warmup", "1", "--no-e2e", "--no-energy",
                        "--no-batch", "--no-serve", "--no-groupby"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["scaling"] in ("weak", "strong") and d["data"] == "synthetic"
    assert d["vs_baseline"] is None and d["unit"] == "GB/s" and "workload" in d["config"]
    assert d["value"] > 0 and d["ms_per_step"] > 0
    # value is the step's bytes over the step time
    assert abs(d["value"] * 1e9 * d["ms_per_step"] * 1e-3 / d["config"]["bytes_per_step"] - 1) < 0.01
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert 0 < rf["achieved"] <= rf["peak"] * 1.05
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert rf["traffic"] is None or rf["traffic"] >= rf["algorithmic_bytes_per_launch"]
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["unit"] == "GB/s"


def test_energy_power_from_counter_updates():
    bench = load_bench()
    res = 15.3                     # microjoules per count
    per_s = 500.0 / (res * 1e-6)   # counts per second at 500 W
    # updates once a second for 5 s
    edges = [(10.0 + i, 1_000_000 + int(i * per_s)) for i in range(6)]
    w, info = bench.energy_power(edges, 9.5, 16.0, res)
    assert abs(w - 500.0) < 0.01 and info["intervals_used"] == 5 and info["intervals_rejected"] == 0
    # updates outside the window do not count
    w2, _ = bench.energy_power(edges + [(30.0, 10 ** 12)], 9.5, 16.0, res)
    assert w2 == w


def test_energy_power_rejects_close_updates_and_misreads():
    bench = load_bench()
    res = 15.3
    # two updates milliseconds apart: too short a span, no value
    w, info = bench.energy_power([(1.0, 100), (1.002, 100 + 65_000)], 0.0, 5.0, res)
    assert w is None and "span" in info["reason"]
    # a single update: no interval at all
    w, info = bench.energy_power([(1.0, 100)], 0.0, 5.0, res)
    assert w is None and "fewer than 2" in info["reason"]
    # a misread (the counter jumps to a huge value, then back, then on): the
    # two bad intervals are dropped with their time, the rest gives 300 W
    per_s = 300.0 / (res * 1e-6)
    good = [(float(i), int(i * per_s)) for i in range(8)]
    bad = good[:3] + [(2.5, 2 ** 50)] + good[3:]
    w, info = bench.energy_power(bad, -1.0, 10.0, res)
    assert abs(w - 300.0) < 0.01 and info["intervals_rejected"] == 2
    # a counter that goes backwards (wrap or reset) and then continues
    wrap = good[:4] + [(4.0, 5)] + [(5.0 + i, 5 + int((i + 1) * per_s)) for i in range(3)]
    w, info = bench.energy_power(wrap, -1.0, 10.0, res)
    assert abs(w - 300.0) < 0.01 and info["intervals_rejected"] == 1
    # an implausible average (every interval a jump) gives no value
    w, info = bench.energy_power([(float(i), i * 10 ** 12) for i in range(5)], -1.0, 10.0, res)
    assert w is None
