"""GPU: many columns in one persistent launch under a HIP graph (agg_batch).

Each batch result must equal the same column's agg_run result bit for bit
(one canonical reduction shape per column) and the oracle; graph replays are
interleaved with eager work and each is checked; launch parameters (retune,
autotune) must not change a bit; the graph reads the columns' current
contents on every replay.
"""
import numpy as np
import pytest

import datagen
from aggcheck import check, same_bits

pytestmark = pytest.mark.gpu

DTS = ["i32", "i64", "f32"]
OPS = ["sum", "min", "max", "avg", "count"]
PRECS = ["neumaier", "f32", "f64_combine"]
TORCH_DT = None


@pytest.fixture(scope="module")
def agg():
    import torch
    import paper_2606_10030_amd as agg
    assert torch.cuda.is_available()
    return agg


def make_columns(seed: int, ncols: int, max_len: int):
    """Mixed columns: log-uniform lengths (with empties), random dtype / op /
    precision, some at unaligned addresses inside a larger buffer."""
    import torch
    r = np.random.default_rng(seed)
    cols = []
    for i in range(ncols):
        dt = DTS[r.integers(0, 3)]
        op = OPS[r.integers(0, 5)]
        prec = PRECS[r.integers(0, 3)] if dt == "f32" else "neumaier"
        n = 0 if r.random() < 0.03 else int(np.exp(r.uniform(0, np.log(max_len))))
        off = int(r.integers(0, 4)) if r.random() < 0.3 else 0
        if dt == "f32" and r.random() < 0.5:
            x = (r.standard_normal(n + off) * np.exp2(r.integers(-20, 21, size=n + off))).astype(np.float32)
        else:
            x = datagen.column(n + off, dt, "uniform", seed=int(seed * 10000 + i))
        d = torch.from_numpy(x).to("cuda")[off:off + n]
        cols.append(dict(x=x[off:off + n], d=d, dtype=dt, op=op, prec=prec))
    return cols


def batch_of(agg, cols, tune=None):
    return agg.Batch([agg.BatchColumn(c["d"], c["op"], c["prec"]) for c in cols], tune=tune)


def singles(agg, cols):
    out = []
    for c in cols:
        p = agg.Plan(c["dtype"], c["op"], max_n=max(1, c["x"].size), prec=c["prec"])
        out.append(p.run(c["d"], n=c["x"].size))
        p.close()
    return out


def test_batch_matches_single_runs_and_oracle(agg):
    cols = make_columns(1, 300, 3_000_000)
    b = batch_of(agg, cols)
    got = b.run()
    ref = singles(agg, cols)
    for i, (c, g, s) in enumerate(zip(cols, got, ref)):
        assert same_bits(g, s), f"column {i} ({c['dtype']} {c['op']} {c['prec']} n={c['x'].size}): batch != agg_run"
        check(c["x"], c["dtype"], c["op"], c["prec"], g, ctx=f"batch col {i}")
    info = b.info()
    assert info["nitems"] > 0 and info["nseg_total"] >= sum(1 for c in cols if c["x"].size)


def test_graph_replays_interleaved_with_eager_work(agg):
    import torch
    cols = make_columns(2, 120, 1_000_000)
    b = batch_of(agg, cols)
    ref = singles(agg, cols)
    out = torch.zeros(len(cols) * 32, dtype=torch.uint8, device="cuda")
    for rep in range(5):
        out.zero_()
        b.enqueue(out)
        # eager work on the same stream between replays
        z = agg.Plan("i64", "sum", max_n=1000)
        assert z.run(torch.arange(1000, dtype=torch.int64, device="cuda"))["i64"] == 499500
        z.close()
        torch.cuda.synchronize()
        got = agg.parse_results(out.cpu().numpy().tobytes(), b.kinds)
        for i, (g, s) in enumerate(zip(got, ref)):
            assert same_bits(g, s), f"replay {rep} column {i}"


def test_launch_parameters_do_not_change_batch_bits(agg):
    cols = make_columns(3, 150, 2_000_000)
    b = batch_of(agg, cols)
    ref = b.run()
    for u, w, bp in [(4, 1, 1), (8, 4, 2), (16, 2, 1), (32, 2, 1), (16, 16, 2), (8, 8, 8)]:
        b.retune(agg.make_tune(unroll=u, waves_per_block=w, blocks_per_cu=bp))
        got = b.run()
        for i, (g, s) in enumerate(zip(got, ref)):
            assert same_bits(g, s), f"tune u{u} w{w} b{bp}: column {i} differs"
    t, ms = b.autotune()
    assert ms > 0 and t.unroll in (4, 8, 16)  # the batch autotuner's candidates (32 spills registers)
    got = b.run()
    for g, s in zip(got, ref):
        assert same_bits(g, s)


def test_batch_reads_current_contents(agg):
    import torch
    cols = make_columns(4, 40, 500_000)
    b = batch_of(agg, cols)
    b.run()
    for c in cols:  # overwrite every column in place
        if c["x"].size:
            c["d"].mul_(-1) if c["dtype"] != "i32" else c["d"].sub_(7)
    torch.cuda.synchronize()
    got = b.run()
    for i, (c, g) in enumerate(zip(cols, got)):
        x = c["d"].cpu().numpy()
        check(x, c["dtype"], c["op"], c["prec"], g, ctx=f"updated col {i}")


def test_empty_and_tiny_batches(agg):
    import torch
    b = agg.Batch([])
    assert b.run() == []
    one = torch.tensor([5], dtype=torch.int32, device="cuda")
    b = agg.Batch([agg.BatchColumn(one, "max"), agg.BatchColumn(one[:0], "min"), agg.BatchColumn(one, "count")])
    r = b.run()
    assert r[0]["value"] == 5 and r[1]["is_null"] and r[2]["value"] == 1
