"""The C-ABI library without a GPU: it loads, exports every declared symbol,
computes canonical shapes on the host, and rejects bad arguments (or reports
no device) cleanly, without touching a kernel."""
import ctypes
import os
import subprocess

import pytest

import paper_2606_10030_amd as agg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(agg.LIB_PATH):
        agg.build()
    return agg.lib()


def test_exports_every_declared_symbol(L):
    declared = agg.declared_symbols()
    assert "agg_run" in declared and "agg_batch_plan" in declared and len(declared) >= 13
    out = subprocess.run(["nm", "-D", "--defined-only", agg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in declared if s not in exported]
    assert not missing, f"declared in agg.h but not exported: {missing}"
    for s in declared:
        assert hasattr(L, s)


def test_library_carries_gfx950_device_code(L):
    sec = subprocess.run(["readelf", "-S", agg.LIB_PATH], capture_output=True, text=True).stdout
    assert ".hip_fatbin" in sec
    # the offload bundle names its target
    assert b"amdgcn-amd-amdhsa--gfx950" in open(agg.LIB_PATH, "rb").read()


@pytest.mark.parametrize("dtype,w", [("i32", 4), ("i64", 8), ("f32", 4)])
def test_canonical_shape_rules(dtype, w):
    prev = None
    for n in [0, 1, 3, 4095, 4096, 4097, 2**20, 2**20 + 13, 10**7, 2**30, 2**31 + 5, 2**33]:
        s = agg.canonical_shape(dtype, n)
        assert s.width == w
        assert s.seg_bytes >= 16 * 1024 and (s.seg_bytes & (s.seg_bytes - 1)) == 0
        assert s.elems_per_seg * w == s.seg_bytes
        assert s.nseg <= 8192
        assert (s.nseg - 1) * s.seg_bytes < n * w <= s.nseg * s.seg_bytes or (n == 0 and s.nseg == 0)
        if prev is not None:
            assert s.seg_bytes >= prev.seg_bytes  # monotone in n
        prev = s
    assert agg.canonical_shape(dtype, 2**30).nseg == 8192


def test_canonical_shape_rejects_bad_args(L):
    s = agg.Shape()
    assert L.agg_canonical_shape(7, 10, ctypes.byref(s)) == agg.E_INVALID
    assert L.agg_canonical_shape(0, -1, ctypes.byref(s)) == agg.E_INVALID
    assert L.agg_canonical_shape(0, 10, None) == agg.E_INVALID


def test_strerror_and_default_tune(L):
    for code in (agg.OK, agg.E_INVALID, agg.E_NOMEM, agg.E_NODEVICE, agg.E_HIP, -99):
        assert isinstance(agg.strerror(code), str) and agg.strerror(code)
    t = agg.default_tune("f32", "sum", 2**30)
    assert t.waves_per_block in (4, 8, 16) and t.unroll in (4, 8, 16)
    assert t.staging_depth in (2, 3, 4) and t.chunk_bytes >= 1 << 20
    bad = agg.Tune()
    assert L.agg_default_tune(0, 9, 0, 10, 0, ctypes.byref(bad)) == agg.E_INVALID


def test_invalid_arguments_are_rejected_before_any_device_work(L):
    h = ctypes.c_void_p()
    assert L.agg_plan(None, 0, 0, 0, 10, 0, None) == agg.E_INVALID
    assert L.agg_plan(ctypes.byref(h), 5, 0, 0, 10, 0, None) == agg.E_INVALID      # dtype
    assert L.agg_plan(ctypes.byref(h), 0, 9, 0, 10, 0, None) == agg.E_INVALID      # op
    assert L.agg_plan(ctypes.byref(h), 2, 0, 7, 10, 0, None) == agg.E_INVALID      # prec for f32 sum
    assert L.agg_plan(ctypes.byref(h), 0, 0, 0, -1, 0, None) == agg.E_INVALID      # max_n
    assert L.agg_plan(ctypes.byref(h), 0, 0, 0, 10, 9, None) == agg.E_INVALID      # src
    bad = agg.make_tune(unroll=5)
    assert L.agg_plan(ctypes.byref(h), 0, 0, 0, 10, 0, ctypes.byref(bad)) == agg.E_INVALID
    bad = agg.make_tune(waves_per_block=3)
    assert L.agg_plan(ctypes.byref(h), 0, 0, 0, 10, 0, ctypes.byref(bad)) == agg.E_INVALID
    assert L.agg_run(None, None, 0, None, None) == agg.E_INVALID
    assert L.agg_plan_destroy(None) == agg.E_INVALID
    assert L.agg_batch_run(None, None, None) == agg.E_INVALID
    assert L.agg_batch_destroy(None) == agg.E_INVALID
    col = agg.Col(None, 5, 0, 0, 0, 0)  # null pointer with n > 0
    assert L.agg_batch_plan(ctypes.byref(h), ctypes.byref(col), 1, None) == agg.E_INVALID


def test_no_device_is_reported_cleanly(L):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    assert L.agg_init(0) == agg.E_NODEVICE
    assert L.agg_plan(ctypes.byref(h), 0, 0, 0, 10, 0, None) == agg.E_NODEVICE
    assert not h.value
    with pytest.raises(agg.AggError):
        agg.Plan("i32", "sum", 10)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(agg, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(agg, "_lib_handle", None)
    with pytest.raises(agg.AggError):
        agg.lib()
