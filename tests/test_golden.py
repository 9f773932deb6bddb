"""Hand-derived fixtures (tests/golden/closed_forms.json) against the oracle
(CPU) and against the HIP path (GPU).

Every expected value in the fixture is a closed form or an IEEE-754 rule,
stated beside it; none was produced by code."""
import json
import math
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
FIX = json.load(open(os.path.join(HERE, "golden", "closed_forms.json")))
NP = {"i32": np.int32, "i64": np.int64, "f32": np.float32}


def column(case):
    dt = NP[case["dtype"]]
    if "arange" in case:
        return np.arange(*case["arange"], dtype=dt)
    if "repeat" in case:
        items, times = case["repeat"]
        return np.tile(np.array([float(v) if isinstance(v, str) else v for v in items], dtype=dt), times)
    return np.array([float(v) if isinstance(v, str) else v for v in case["values"]], dtype=dt)


def check(got_i64, got_f64, got_null, want, ctx):
    if want is None:
        assert got_null, f"{ctx}: expected no value"
        return
    assert not got_null, f"{ctx}: unexpected null"
    if "i64" in want:
        assert got_i64 == want["i64"], f"{ctx}: {got_i64} != {want['i64']}"
    else:
        w = float(want["f64"])
        assert (math.isnan(w) and math.isnan(got_f64)) or got_f64 == w, f"{ctx}: {got_f64!r} != {w!r}"


@pytest.mark.parametrize("case", FIX["cases"], ids=[c["name"] for c in FIX["cases"]])
def test_oracle_matches_closed_forms(case):
    x = column(case)
    for op, want in case["expect"].items():
        r = oracle.aggregate(x, op)
        check(r.i64, r.f64, r.is_null, want, f"{case['name']} {op}")


@pytest.mark.parametrize("case", FIX["groupby"], ids=[c["name"] for c in FIX["groupby"]])
def test_oracle_groupby_matches_closed_forms(case):
    keys = np.array(case["keys"], NP[case["key_dtype"]])
    vals = np.array(case["vals"], NP[case["val_dtype"]])
    for op, want in case["expect"].items():
        got = [(k, i, c) for k, i, _, c in oracle.groupby(keys, vals, op)]
        assert got == [tuple(w) for w in want], f"{case['name']} {op}: {got}"


@pytest.mark.gpu
def test_hip_path_matches_closed_forms():
    import torch
    import paper_2606_10030_amd as agg
    for case in FIX["cases"]:
        x = column(case)
        dev = torch.from_numpy(x).to("cuda")
        for op, want in case["expect"].items():
            r = agg.Plan(case["dtype"], op, max_n=max(x.size, 1)).run(dev)
            if op in case.get("gpu_non_finite", []):
                # float32 lane accumulators overflow past FLT_MAX (documented)
                assert not math.isfinite(r["f64"]), f"{case['name']} {op}: {r['f64']!r}"
                continue
            check(r["i64"], r["f64"], r["is_null"], want, f"{case['name']} {op}")
    for case in FIX["groupby"]:
        keys = torch.tensor(case["keys"], dtype={"i32": torch.int32, "i64": torch.int64}[case["key_dtype"]], device="cuda")
        vals = torch.tensor(case["vals"], dtype={"i32": torch.int32, "i64": torch.int64}[case["val_dtype"]], device="cuda")
        for op, want in case["expect"].items():
            g = agg.GroupBy(case["key_dtype"], case["val_dtype"], op, max_n=keys.numel(), max_groups=8)
            got = [(k, i, c) for k, i, _, c in g.run(keys, vals)]
            assert got == [tuple(w) for w in want], f"{case['name']} {op}: {got}"
