"""The packed int32 format: the host encoder against an independent decoder
written from the layout documented in agg.h (CPU only)."""
import numpy as np
import pytest

import datagen
import paper_2606_10030_amd as agg


def decode(pc: agg.PackedColumn) -> np.ndarray:
    """Plain decoder of the documented layout."""
    out = np.empty(pc.n, dtype=np.int64)
    for b, h in enumerate(pc.blocks):
        bits, base, off = int(h["bits"]), int(h["base"]), int(h["word_off"])
        for lane in range(64):
            words = [int(pc.payload[off + j * 64 + lane]) for j in range(bits)]
            stream = sum(w << (32 * j) for j, w in enumerate(words))
            for i in range(32):
                idx = b * 2048 + lane * 32 + i
                if idx >= pc.n:
                    break
                d = (stream >> (i * bits)) & ((1 << bits) - 1)
                v = (base + d) & 0xFFFFFFFF
                out[idx] = v - (1 << 32) if v >= 1 << 31 else v
    return out


@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 2047, 2048, 2049, 10_000])
def test_round_trip_uniform(n):
    x = datagen.column(n, "i32", "uniform", seed=n + 1)
    pc = agg.pack_i32(x, threads=3)
    assert pc.n == n and len(pc.blocks) == -(-n // 2048)
    assert np.array_equal(decode(pc), x.astype(np.int64))
    if n:
        assert all(h["bits"] <= 21 for h in pc.blocks)   # range 2^21
        assert pc.payload_words == sum(64 * int(h["bits"]) for h in pc.blocks)


def test_round_trip_edge_widths():
    r = np.random.default_rng(0)
    cols = {
        "constant": np.full(5000, -7, np.int32),                                   # bits 0
        "binary": r.integers(0, 2, 5000).astype(np.int32),                          # bits 1
        "full_range": r.integers(-2**31, 2**31, 5000, dtype=np.int64).astype(np.int32),  # bits 32
        "extremes": np.array([-2**31, 2**31 - 1] * 1500, np.int32),
        "sorted": np.sort(r.integers(-10**9, 10**9, 6000)).astype(np.int32),
        "span31": np.array([0, 2**31 - 1, 5, 9] * 1000, np.int32),
    }
    for name, x in cols.items():
        pc = agg.pack_i32(x)
        assert np.array_equal(decode(pc), x.astype(np.int64)), name
    assert all(h["bits"] == 0 for h in agg.pack_i32(cols["constant"]).blocks)
    assert all(h["bits"] == 32 for h in agg.pack_i32(cols["extremes"]).blocks)


def test_thread_count_does_not_change_the_encoding():
    x = datagen.column(300_001, "i32", "zipf", seed=3)
    a, b = agg.pack_i32(x, threads=1), agg.pack_i32(x, threads=7)
    assert a.payload_words == b.payload_words
    assert np.array_equal(a.payload, b.payload) and a.blocks.tobytes() == b.blocks.tobytes()


def test_compression_ratio_of_key_columns():
    x = datagen.column(1 << 20, "i32", "uniform", seed=5, lo=1, hi=2_000_001)   # SF200-like keys
    pc = agg.pack_i32(x)
    ratio = pc.nbytes / (4 * x.size)
    assert 0.65 < ratio < 0.68        # 21 of 32 bits plus a 16-byte header per 2048 items
    s = datagen.column(1 << 20, "i32", "sorted", seed=5)
    assert agg.pack_i32(s).nbytes < 0.42 * 4 * s.size   # 2048 sorted values span about 2^12
