"""GPU: the autotuner and its cache.  Tuning changes speed, never bits."""
import json

import numpy as np
import pytest

import oracle
from aggcheck import check, same_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    agg.tune_clear()
    yield agg
    agg.tune_clear()


def test_autotune_picks_valid_parameters_and_keeps_bits(agg, tmp_path):
    import torch
    r = np.random.default_rng(0)
    x = (r.standard_normal(1 << 25) * np.exp2(r.integers(-20, 21, size=1 << 25))).astype(np.float32)
    d = torch.from_numpy(x).to("cuda")
    before = agg.Plan("f32", "sum", max_n=x.size).run(d)
    t, gbs = agg.autotune("f32", "sum", d)
    assert gbs > 100 and t.unroll in (8, 16, 32) and t.waves_per_block in (1, 2, 4, 8)
    # plans without explicit parameters now use the cache entry
    dt = agg.default_tune("f32", "sum", x.size)
    assert dt.as_dict() == t.as_dict()
    after = agg.Plan("f32", "sum", max_n=x.size).run(d)
    assert same_bits(before, after)
    check(x, "f32", "sum", "neumaier", after, ctx="autotuned")
    # save / load round trip
    path = str(tmp_path / "tune.json")
    agg.tune_save(path)
    doc = json.load(open(path))
    assert doc["version"] == 1 and doc["device"].startswith("gfx950") and len(doc["entries"]) == 1
    agg.tune_clear()
    agg.tune_load(path)
    assert agg.default_tune("f32", "sum", x.size).as_dict() == t.as_dict()


def test_tune_load_rejects_other_devices_and_garbage(agg, tmp_path):
    p = tmp_path / "other.json"
    p.write_text(json.dumps({"version": 1, "device": "gfx942/304", "entries": []}))
    with pytest.raises(agg.AggError):
        agg.tune_load(str(p))
    g = tmp_path / "garbage.json"
    g.write_text("{not json")
    with pytest.raises(agg.AggError):
        agg.tune_load(str(g))
    with pytest.raises(agg.AggError):
        agg.tune_load(str(tmp_path / "missing.json"))


def test_autotune_pinned_host_source(agg):
    import torch
    x = torch.randint(-2**20, 2**20, (1 << 26,), dtype=torch.int32).pin_memory()
    t, gbs = agg.autotune("i32", "sum", x, src="pinned_host")
    assert gbs > 1 and t.staging_depth in (2, 3, 4) and t.chunk_bytes >= 16 << 20
    got = agg.Plan("i32", "sum", max_n=x.numel(), src="pinned_host").run(x)
    assert got["i64"] == oracle.value(x.numpy(), "sum")
