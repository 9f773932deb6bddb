"""MI355X (gfx950) in-memory aggregation scan: Python binding of libagg.so.

This module only marshals arguments to the C ABI declared in
``include/agg.h``; every step of the scan runs in the HIP kernels of the
library.  PyTorch is used for device memory, pinned host memory and streams.
There is no fallback: if ``libagg.so`` is missing or fails to load, every call
raises ``AggError``.

    import torch, paper_2606_10030_amd as agg
    x = torch.randint(-2**20, 2**20, (1 << 20,), dtype=torch.int32, device="cuda")
    plan = agg.Plan("i32", "sum", max_n=x.numel())
    print(plan.run(x)["i64"])
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass
from typing import Iterable, Optional, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libagg.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "agg.h")

OK, E_INVALID, E_NOMEM, E_NODEVICE, E_HIP = 0, -1, -2, -3, -4
I32, I64, F32 = 0, 1, 2
SUM, MIN, MAX, COUNT, AVG = 0, 1, 2, 3, 4
PREC_NEUMAIER, PREC_F32, PREC_F64_COMBINE = 0, 1, 2
SRC_DEVICE, SRC_PINNED_HOST, SRC_ZEROCOPY = 0, 1, 2

DTYPES = {"i32": I32, "i64": I64, "f32": F32}
OPS = {"sum": SUM, "min": MIN, "max": MAX, "count": COUNT, "avg": AVG}
PRECS = {"neumaier": PREC_NEUMAIER, "f32": PREC_F32, "f64_combine": PREC_F64_COMBINE}
SRCS = {"device": SRC_DEVICE, "pinned_host": SRC_PINNED_HOST, "zerocopy": SRC_ZEROCOPY}
WIDTH = {I32: 4, I64: 8, F32: 4}


class AggError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if _lib_handle else f"{what} ({code})")


class Result(ctypes.Structure):
    _fields_ = [("i64", ctypes.c_int64), ("f64", ctypes.c_double), ("count", ctypes.c_int64),
                ("is_null", ctypes.c_int32), ("prec_used", ctypes.c_int32)]


class Tune(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("chunk_bytes", ctypes.c_int64), ("staging_depth", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Shape(ctypes.Structure):
    _fields_ = [("seg_bytes", ctypes.c_int64), ("nseg", ctypes.c_int64),
                ("elems_per_seg", ctypes.c_int64), ("width", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Col(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("n", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("op", ctypes.c_int32), ("prec", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("n", ctypes.c_int64), ("column_id", ctypes.c_int64),
                ("arrival_s", ctypes.c_double), ("dtype", ctypes.c_int32), ("op", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("resident", ctypes.c_int32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("cache_shipped", ctypes.c_int32), ("chunk_bytes", ctypes.c_int64),
                ("max_shipping", ctypes.c_int32), ("progress_every", ctypes.c_int32)]


class RequestStats(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("bytes_shipped", ctypes.c_int64), ("slot", ctypes.c_int32), ("status", ctypes.c_int32),
                ("cache_hit", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServeSummary(ctypes.Structure):
    _fields_ = [("makespan_s", ctypes.c_double), ("bytes_scanned", ctypes.c_int64),
                ("bytes_shipped", ctypes.c_int64), ("peak_reserved_bytes", ctypes.c_int64),
                ("peak_busy_slots", ctypes.c_int32), ("completed", ctypes.c_int32),
                ("failed", ctypes.c_int32), ("cache_hits", ctypes.c_int32)]


def _struct_dict(x) -> dict:
    return {f: getattr(x, f) for f, _ in x._fields_ if f != "reserved"}


class Filter(ctypes.Structure):
    _fields_ = [("col", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("lo_inclusive", ctypes.c_int32),
                ("hi_inclusive", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ilo", ctypes.c_int64),
                ("ihi", ctypes.c_int64), ("flo", ctypes.c_double), ("fhi", ctypes.c_double)]


def make_filter(col, lo=None, hi=None, lo_inclusive: bool = True, hi_inclusive: bool = True,
                dtype=None) -> Filter:
    """A range predicate lo <=/< y <=/< hi on the filter column `col` (a device
    tensor, or an int address with `dtype`); a missing bound is open."""
    if isinstance(col, int):
        ptr, dt = col, _code(dtype, DTYPES, "dtype")
    else:
        ptr, dt = col.data_ptr(), _dtype_of_tensor(col)
    inf = float("inf")
    if dt == F32:
        flo = -inf if lo is None else float(lo)
        fhi = inf if hi is None else float(hi)
        return Filter(ptr, dt, 1 if lo is None else int(lo_inclusive), 1 if hi is None else int(hi_inclusive),
                      0, 0, 0, flo, fhi)
    ilo = -(1 << 63) if lo is None else int(lo)
    ihi = (1 << 63) - 1 if hi is None else int(hi)
    return Filter(ptr, dt, 1 if lo is None else int(lo_inclusive), 1 if hi is None else int(hi_inclusive), 0,
                  ilo, ihi, 0.0, 0.0)


class Packed(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_void_p), ("payload", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("payload_words", ctypes.c_int64), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


PACK_BLOCK = 2048
RESULT_BYTES = ctypes.sizeof(Result)
assert RESULT_BYTES == 32

_lib_handle = None


def build() -> str:
    """Compile libagg.so in-tree with hipcc for gfx950."""
    from ._build import build as _b
    global _lib_handle
    _lib_handle = None
    return _b()


def lib():
    """The loaded library; raises AggError if it is not built."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise AggError(E_NODEVICE, f"libagg.so not built at {LIB_PATH}; call paper_2606_10030_amd.build()")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "agg_init": ([i32], ctypes.c_int),
        "agg_device_info": ([i32, ctypes.POINTER(i32), ctypes.c_char_p, i32], ctypes.c_int),
        "agg_canonical_shape": ([i32, i64, ctypes.POINTER(Shape)], ctypes.c_int),
        "agg_default_tune": ([i32, i32, i32, i64, i32, ctypes.POINTER(Tune)], ctypes.c_int),
        "agg_plan": ([ctypes.POINTER(vp), i32, i32, i32, i64, i32, ctypes.POINTER(Tune)], ctypes.c_int),
        "agg_run": ([vp, vp, i64, vp, vp], ctypes.c_int),
        "agg_run_noalloc": ([i32, i32, i32, i32, vp, i64, vp, vp], ctypes.c_int),
        "agg_plan_info": ([vp, i64, ctypes.POINTER(Shape), ctypes.POINTER(Tune)], ctypes.c_int),
        "agg_plan_destroy": ([vp], ctypes.c_int),
        "agg_batch_plan": ([ctypes.POINTER(vp), ctypes.POINTER(Col), i32, ctypes.POINTER(Tune)], ctypes.c_int),
        "agg_batch_run": ([vp, vp, vp], ctypes.c_int),
        "agg_batch_destroy": ([vp], ctypes.c_int),
        "agg_batch_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(Tune)], ctypes.c_int),
        "agg_batch_retune": ([vp, ctypes.POINTER(Tune)], ctypes.c_int),
        "agg_batch_autotune": ([vp, vp, ctypes.POINTER(Tune), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "agg_autotune": ([i32, i32, i32, vp, i64, i32, vp, ctypes.POINTER(Tune), ctypes.POINTER(ctypes.c_double)],
                         ctypes.c_int),
        "agg_tune_save": ([ctypes.c_char_p], ctypes.c_int),
        "agg_tune_load": ([ctypes.c_char_p], ctypes.c_int),
        "agg_tune_clear": ([], ctypes.c_int),
        "agg_serve_create": ([ctypes.POINTER(vp), ctypes.POINTER(ServeConfig)], ctypes.c_int),
        "agg_serve_run": ([vp, ctypes.POINTER(Request), i32, vp, ctypes.POINTER(RequestStats),
                           ctypes.POINTER(ServeSummary)], ctypes.c_int),
        "agg_serve_destroy": ([vp], ctypes.c_int),
        "agg_serve_simulate": ([ctypes.POINTER(ServeConfig), ctypes.POINTER(Request), i32, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.POINTER(RequestStats),
                                ctypes.POINTER(ServeSummary)], ctypes.c_int),
        "agg_run_filtered": ([vp, vp, i64, ctypes.POINTER(Filter), vp, vp], ctypes.c_int),
        "agg_groupby_plan": ([ctypes.POINTER(vp), i32, i32, i32, i64, i64], ctypes.c_int),
        "agg_groupby_run": ([vp, vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "agg_groupby_destroy": ([vp], ctypes.c_int),
        "agg_pack_bound": ([i64, ctypes.POINTER(i64)], ctypes.c_int),
        "agg_pack_i32": ([vp, i64, vp, vp, i64, ctypes.POINTER(i64), i32], ctypes.c_int),
        "agg_run_packed": ([vp, ctypes.POINTER(Packed), vp, vp], ctypes.c_int),
        "agg_fault_inject": ([i32, i32], ctypes.c_int),
        "agg_strerror": ([i32], ctypes.c_char_p),
        "agg_last_hip_error": ([], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib_handle = L
    return L


def declared_symbols() -> list:
    """Every function declared in include/agg.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(agg_\w+)\s*\(", text, re.M)))


FAULT_SITES = {"alloc": 1, "ship": 2}


def fault_inject(site, countdown: int) -> None:
    """Make the countdown-th next event at `site` ("alloc": a library
    allocation -> AGG_E_NOMEM; "ship": a shipped serving copy -> AGG_E_HIP for
    that request) fail; 0 disarms it (agg_fault_inject)."""
    _check(lib().agg_fault_inject(_code(site, FAULT_SITES, "fault site"), int(countdown)), "agg_fault_inject")


def strerror(code: int) -> str:
    return lib().agg_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != OK:
        if rc == E_HIP:
            raise AggError(rc, f"{what} (hipError {lib().agg_last_hip_error()})")
        raise AggError(rc, what)


def _code(v, table, what):
    if isinstance(v, str):
        if v not in table:
            raise ValueError(f"unknown {what} {v!r}")
        return table[v]
    return int(v)


def _torch():
    import torch
    return torch


_TENSOR_DTYPES = None


def _dtype_of_tensor(t) -> int:
    global _TENSOR_DTYPES
    if _TENSOR_DTYPES is None:
        torch = _torch()
        _TENSOR_DTYPES = {torch.int32: I32, torch.int64: I64, torch.float32: F32}
    code = _TENSOR_DTYPES.get(t.dtype)
    if code is None:
        raise TypeError(f"unsupported column dtype {t.dtype}")
    return code


def _stream_handle(stream) -> int:
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def canonical_shape(dtype, n: int) -> Shape:
    s = Shape()
    _check(lib().agg_canonical_shape(_code(dtype, DTYPES, "dtype"), n, ctypes.byref(s)), "agg_canonical_shape")
    return s


def float_sum_bound_coeff(prec, n: int) -> float:
    """The documented a-priori bound of a float32 SUM over n items in precision
    mode `prec`, as a multiple of sum |x| (include/agg.h): with u = 2^-24,
    v = 2^-53, m = seg_bytes / 1024 and k = ceil(nseg / 256) of the canonical
    shape, gamma_d(w) = d w / (1 - d w):
    compensated 1.01 ((44 ceil(m/8) + 24) u^2 + (k + 8) v); plain
    gamma_{m+k+18}(u); f64-combine gamma_{m+8}(u) + gamma_{k+8}(v) (1 + gamma_{m+8}(u))."""
    p = _code(prec, PRECS, "prec")
    s = canonical_shape(F32, n)
    m = s.seg_bytes // 1024
    k = -(-s.nseg // 256)
    u, v = 2.0 ** -24, 2.0 ** -53

    def gamma(d, w):
        return d * w / (1.0 - d * w)
    if p == PREC_F32:
        return gamma(m + k + 18, u)
    if p == PREC_F64_COMBINE:
        g = gamma(m + 8, u)
        return g + gamma(k + 8, v) * (1.0 + g)
    return 1.01 * ((44 * -(-m // 8) + 24) * u * u + (k + 8) * v)


def default_tune(dtype, op, n: int, prec="neumaier", src="device") -> Tune:
    t = Tune()
    _check(lib().agg_default_tune(_code(dtype, DTYPES, "dtype"), _code(op, OPS, "op"),
                                  _code(prec, PRECS, "prec"), n, _code(src, SRCS, "src"),
                                  ctypes.byref(t)), "agg_default_tune")
    return t


def make_tune(**kw) -> Tune:
    """A Tune from the built-in defaults with the given fields replaced."""
    t = default_tune("i32", "sum", 1)
    for k, v in kw.items():
        if not hasattr(t, k):
            raise ValueError(f"unknown tune field {k}")
        setattr(t, k, v)
    return t


def autotune(dtype, op, col, n: Optional[int] = None, prec="neumaier", src="device", stream=None):
    """Time candidate launch parameters on `col`; the fastest enters the tuning
    cache (used by later plans without explicit parameters).  Returns (Tune, GB/s)."""
    if isinstance(col, int):
        ptr, nn = col, int(n)
    else:
        ptr, nn = col.data_ptr(), col.numel() if n is None else int(n)
    t, g = Tune(), ctypes.c_double()
    _check(lib().agg_autotune(_code(dtype, DTYPES, "dtype"), _code(op, OPS, "op"), _code(prec, PRECS, "prec"),
                              ptr, nn, _code(src, SRCS, "src"), _stream_handle(stream), ctypes.byref(t),
                              ctypes.byref(g)), "agg_autotune")
    return t, g.value


def tune_save(path: str) -> None:
    _check(lib().agg_tune_save(path.encode()), "agg_tune_save")


def tune_load(path: str) -> None:
    _check(lib().agg_tune_load(path.encode()), "agg_tune_load")


def tune_clear() -> None:
    _check(lib().agg_tune_clear(), "agg_tune_clear")


def device_info(device: int = 0) -> dict:
    cu = ctypes.c_int32()
    arch = ctypes.create_string_buffer(64)
    _check(lib().agg_device_info(device, ctypes.byref(cu), arch, 64), "agg_device_info")
    return {"cu_count": cu.value, "arch": arch.value.decode()}


def result_dict(r: Result, dtype: int, op: int) -> dict:
    d = {"i64": r.i64, "f64": r.f64, "count": r.count, "is_null": bool(r.is_null), "prec_used": r.prec_used}
    if r.is_null:
        d["value"] = None
    elif op == COUNT or (dtype != F32 and op in (SUM, MIN, MAX)):
        d["value"] = r.i64
    else:
        d["value"] = r.f64
    return d


def parse_results(buf, dtype_ops: Sequence) -> list:
    """Decode a bytes-like buffer of agg_result records."""
    raw = bytes(buf)
    out = []
    for i, (dt, op) in enumerate(dtype_ops):
        r = Result.from_buffer_copy(raw, i * RESULT_BYTES)
        out.append(result_dict(r, dt, op))
    return out


class Plan:
    """agg_plan / agg_run for one (dtype, op, prec, src) and columns of up to max_n items."""

    def __init__(self, dtype, op, max_n: int, prec="neumaier", src="device", tune: Optional[Tune] = None):
        self.dtype = _code(dtype, DTYPES, "dtype")
        self.op = _code(op, OPS, "op")
        self.prec = _code(prec, PRECS, "prec")
        self.src = _code(src, SRCS, "src")
        self.max_n = int(max_n)
        h = ctypes.c_void_p()
        _check(lib().agg_plan(ctypes.byref(h), self.dtype, self.op, self.prec, self.max_n, self.src,
                              ctypes.byref(tune) if tune is not None else None), "agg_plan")
        self._h = h
        self._host_out = None
        self._agg_run = lib().agg_run  # looked up once: enqueue is on the small-call path

    def info(self, n: int):
        s, t = Shape(), Tune()
        _check(lib().agg_plan_info(self._h, n, ctypes.byref(s), ctypes.byref(t)), "agg_plan_info")
        return s, t

    def _col_args(self, col, n):
        if isinstance(col, int):
            if n is None:
                raise ValueError("n is required with a raw pointer")
            return col, int(n)
        dt = _dtype_of_tensor(col)
        if dt != self.dtype:
            raise TypeError(f"column dtype {col.dtype} does not match the plan")
        if not col.is_contiguous():
            raise ValueError("column must be contiguous")
        return col.data_ptr(), col.numel() if n is None else int(n)

    def enqueue(self, col, out, n: Optional[int] = None, stream=None) -> None:
        """Enqueue agg_run writing the 32-byte result to `out` (tensor or address); no sync."""
        ptr, nn = self._col_args(col, n)
        optr = out if isinstance(out, int) else out.data_ptr()
        rc = self._agg_run(self._h, ptr, nn, optr, _stream_handle(stream))
        if rc != OK:
            _check(rc, "agg_run")

    def run(self, col, n: Optional[int] = None, stream=None) -> dict:
        """Run and wait; returns the decoded result."""
        torch = _torch()
        if self._host_out is None:
            self._host_out = torch.zeros(RESULT_BYTES, dtype=torch.uint8, pin_memory=True)
        s = _torch().cuda.current_stream() if stream is None else stream
        self.enqueue(col, self._host_out, n=n, stream=s)
        if isinstance(s, int):
            torch.cuda.synchronize()
        else:
            s.synchronize()
        return parse_results(self._host_out.numpy().tobytes(), [(self.dtype, self.op)])[0]

    def enqueue_filtered(self, col, filt: Filter, out, n: Optional[int] = None, stream=None) -> None:
        """Enqueue agg_run_filtered: aggregate the items of `col` selected by `filt`."""
        ptr, nn = self._col_args(col, n)
        optr = out if isinstance(out, int) else out.data_ptr()
        _check(lib().agg_run_filtered(self._h, ptr, nn, ctypes.byref(filt), optr, _stream_handle(stream)),
               "agg_run_filtered")

    def run_filtered(self, col, filt: Filter, n: Optional[int] = None, stream=None) -> dict:
        torch = _torch()
        if self._host_out is None:
            self._host_out = torch.zeros(RESULT_BYTES, dtype=torch.uint8, pin_memory=True)
        s = torch.cuda.current_stream() if stream is None else stream
        self.enqueue_filtered(col, filt, self._host_out, n=n, stream=s)
        s.synchronize()
        return parse_results(self._host_out.numpy().tobytes(), [(self.dtype, self.op)])[0]

    def enqueue_packed(self, packed: "PackedColumn", out, stream=None) -> None:
        """Enqueue agg_run_packed on a PackedColumn in device (src=device) or
        pinned host memory (src=zerocopy)."""
        st = packed.struct()
        optr = out if isinstance(out, int) else out.data_ptr()
        _check(lib().agg_run_packed(self._h, ctypes.byref(st), optr, _stream_handle(stream)), "agg_run_packed")

    def run_packed(self, packed: "PackedColumn", stream=None) -> dict:
        torch = _torch()
        if self._host_out is None:
            self._host_out = torch.zeros(RESULT_BYTES, dtype=torch.uint8, pin_memory=True)
        s = torch.cuda.current_stream() if stream is None else stream
        self.enqueue_packed(packed, self._host_out, stream=s)
        s.synchronize()
        r = parse_results(self._host_out.numpy().tobytes(), [(self.dtype, self.op)])[0]
        if Result.from_buffer_copy(self._host_out.numpy().tobytes()).is_null < 0:
            raise AggError(E_INVALID, "agg_run_packed: corrupt packed block header (result not valid)")
        return r

    def close(self):
        if getattr(self, "_h", None):
            lib().agg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group(ctypes.Structure):
    _fields_ = [("key", ctypes.c_int64), ("i64", ctypes.c_int64), ("f64", ctypes.c_double),
                ("count", ctypes.c_int64)]


GROUP_BYTES = ctypes.sizeof(Group)
assert GROUP_BYTES == 32


class GroupBy:
    """agg_groupby_plan / agg_groupby_run: per-key aggregates of a value column."""

    def __init__(self, key_dtype, val_dtype, op, max_n: int, max_groups: int):
        self.key_dtype = _code(key_dtype, DTYPES, "dtype")
        self.val_dtype = _code(val_dtype, DTYPES, "dtype")
        self.op = _code(op, OPS, "op")
        self.max_n, self.max_groups = int(max_n), int(max_groups)
        h = ctypes.c_void_p()
        _check(lib().agg_groupby_plan(ctypes.byref(h), self.key_dtype, self.val_dtype, self.op, self.max_n,
                                      self.max_groups), "agg_groupby_plan")
        self._h = h
        self._out = None
        self._ng = None

    def _col(self, col, dtype, what):
        if isinstance(col, int):
            return col
        if _dtype_of_tensor(col) != dtype:
            raise TypeError(f"{what} dtype {col.dtype} does not match the plan")
        if not col.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        return col.data_ptr()

    def enqueue(self, keys, vals, groups, ngroups, n: Optional[int] = None, stream=None) -> None:
        """Enqueue agg_groupby_run; `groups` / `ngroups` are tensors or addresses."""
        nn = int(n) if n is not None else keys.numel()
        kp = self._col(keys, self.key_dtype, "keys") if nn else 0
        vp = self._col(vals, self.val_dtype, "values") if nn else 0
        gp = groups if isinstance(groups, int) else groups.data_ptr()
        np_ = ngroups if isinstance(ngroups, int) else ngroups.data_ptr()
        _check(lib().agg_groupby_run(self._h, kp, vp, nn, gp, np_, _stream_handle(stream)), "agg_groupby_run")

    def run(self, keys, vals, n: Optional[int] = None, stream=None):
        """Run and wait; returns [(key, i64, f64, count)] sorted by key, or None
        when the input has more than max_groups distinct keys."""
        torch = _torch()
        if self._out is None:
            self._out = torch.empty(self.max_groups * GROUP_BYTES, dtype=torch.uint8, device="cuda")
            self._ng = torch.zeros(1, dtype=torch.int64, pin_memory=True)
        s = torch.cuda.current_stream() if stream is None else stream
        self.enqueue(keys, vals, self._out, self._ng, n=n, stream=s)
        s.synchronize()
        ng = int(self._ng[0])
        if ng < 0:
            return None
        raw = self._out[:ng * GROUP_BYTES].cpu().numpy().tobytes()
        gs = [Group.from_buffer_copy(raw, i * GROUP_BYTES) for i in range(ng)]
        return sorted(((g.key, g.i64, g.f64, g.count) for g in gs), key=lambda t: t[0])

    def close(self):
        if getattr(self, "_h", None):
            lib().agg_groupby_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class BatchColumn:
    col: object          # torch tensor on the device (or an int address with n and dtype)
    op: object
    prec: object = "neumaier"
    n: Optional[int] = None
    dtype: Optional[object] = None


class Batch:
    """agg_batch_plan / agg_batch_run over many device columns."""

    def __init__(self, columns: Iterable[BatchColumn], tune: Optional[Tune] = None):
        cols = list(columns)
        arr = (Col * max(1, len(cols)))()
        self.kinds = []
        for i, c in enumerate(cols):
            if isinstance(c.col, int):
                ptr, n, dt = c.col, int(c.n), _code(c.dtype, DTYPES, "dtype")
            else:
                ptr, n, dt = c.col.data_ptr(), c.col.numel() if c.n is None else int(c.n), _dtype_of_tensor(c.col)
            op = _code(c.op, OPS, "op")
            arr[i] = Col(ptr, n, dt, op, _code(c.prec, PRECS, "prec"), 0)
            self.kinds.append((dt, op))
        h = ctypes.c_void_p()
        _check(lib().agg_batch_plan(ctypes.byref(h), arr, len(cols),
                                    ctypes.byref(tune) if tune is not None else None), "agg_batch_plan")
        self._h = h
        self.ncols = len(cols)
        self._host_out = None

    def enqueue(self, out, stream=None) -> None:
        optr = out if isinstance(out, int) else out.data_ptr()
        _check(lib().agg_batch_run(self._h, optr, _stream_handle(stream)), "agg_batch_run")

    def info(self) -> dict:
        ni, ns, t = ctypes.c_int64(), ctypes.c_int64(), Tune()
        _check(lib().agg_batch_info(self._h, ctypes.byref(ni), ctypes.byref(ns), ctypes.byref(t)), "agg_batch_info")
        return {"nitems": ni.value, "nseg_total": ns.value, "tune": t.as_dict()}

    def retune(self, tune: Tune) -> None:
        _check(lib().agg_batch_retune(self._h, ctypes.byref(tune)), "agg_batch_retune")

    def autotune(self, stream=None):
        t, ms = Tune(), ctypes.c_double()
        _check(lib().agg_batch_autotune(self._h, _stream_handle(stream), ctypes.byref(t), ctypes.byref(ms)),
               "agg_batch_autotune")
        return t, ms.value

    def run(self, stream=None) -> list:
        torch = _torch()
        if self._host_out is None:
            self._host_out = torch.zeros(max(1, self.ncols) * RESULT_BYTES, dtype=torch.uint8, pin_memory=True)
        s = torch.cuda.current_stream() if stream is None else stream
        self.enqueue(self._host_out, stream=s)
        s.synchronize()
        return parse_results(self._host_out.numpy().tobytes(), self.kinds)

    def close(self):
        if getattr(self, "_h", None):
            lib().agg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
def _requests(reqs) -> "ctypes.Array":
    """Requests from dicts: ptr (int address or tensor), n, column_id, arrival_s,
    dtype, op, prec (default neumaier), resident (bool)."""
    arr = (Request * max(1, len(reqs)))()
    for i, r in enumerate(reqs):
        col = r["ptr"]
        ptr = col if isinstance(col, int) else col.data_ptr()
        n = r["n"] if "n" in r else col.numel()
        arr[i] = Request(ptr, int(n), int(r.get("column_id", i)), float(r["arrival_s"]),
                         _code(r["dtype"], DTYPES, "dtype"), _code(r["op"], OPS, "op"),
                         _code(r.get("prec", "neumaier"), PRECS, "prec"), 1 if r.get("resident") else 0)
    return arr


def _config(hbm_budget_bytes, max_slots, cache_shipped, chunk_bytes, max_shipping, progress_every=0) -> ServeConfig:
    ms = min(int(max_slots), 2) if max_shipping is None else int(max_shipping)
    return ServeConfig(int(hbm_budget_bytes), int(max_slots), 1 if cache_shipped else 0, int(chunk_bytes), ms,
                       int(progress_every))


class Server:
    """agg_serve_create / agg_serve_run: continuous admission of requests on the GPU."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 8, cache_shipped: bool = True,
                 chunk_bytes: int = 64 << 20, max_shipping: Optional[int] = None, progress_every: int = 0):
        self.cfg = _config(hbm_budget_bytes, max_slots, cache_shipped, chunk_bytes, max_shipping, progress_every)
        h = ctypes.c_void_p()
        _check(lib().agg_serve_create(ctypes.byref(h), ctypes.byref(self.cfg)), "agg_serve_create")
        self._h = h

    def run(self, reqs: list):
        """Serve the requests (sorted by arrival_s); returns (results, stats, summary)."""
        arr = _requests(reqs)
        n = len(reqs)
        res = (Result * max(1, n))()
        st = (RequestStats * max(1, n))()
        sm = ServeSummary()
        _check(lib().agg_serve_run(self._h, arr, n, ctypes.cast(res, ctypes.c_void_p), st, ctypes.byref(sm)),
               "agg_serve_run")
        results = [result_dict(res[i], arr[i].dtype, arr[i].op) for i in range(n)]
        return results, [_struct_dict(st[i]) for i in range(n)], _struct_dict(sm)

    def close(self):
        if getattr(self, "_h", None):
            lib().agg_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_simulate(reqs: list, hbm_budget_bytes: int, max_slots: int = 8, cache_shipped: bool = True,
                   chunk_bytes: int = 64 << 20, pcie_gbs: float = 55.0, hbm_gbs: float = 7000.0,
                   launch_s: float = 10e-6, max_shipping: Optional[int] = None):
    """The serving scheduler on the CPU with a simulated clock (no device)."""
    cfg = _config(hbm_budget_bytes, max_slots, cache_shipped, chunk_bytes, max_shipping)
    arr = _requests(reqs)
    n = len(reqs)
    st = (RequestStats * max(1, n))()
    sm = ServeSummary()
    _check(lib().agg_serve_simulate(ctypes.byref(cfg), arr, n, pcie_gbs, hbm_gbs, launch_s, st, ctypes.byref(sm)),
           "agg_serve_simulate")
    return [_struct_dict(st[i]) for i in range(n)], _struct_dict(sm)


def percentile(xs, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(xs)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]


# ------------------------------------------------------------------ packed columns
def _np():
    import numpy as np
    return np


BLOCK_DTYPE = None


def block_dtype():
    global BLOCK_DTYPE
    if BLOCK_DTYPE is None:
        np = _np()
        BLOCK_DTYPE = np.dtype([("base", "<i4"), ("bits", "<u4"), ("word_off", "<i8")])
    return BLOCK_DTYPE


@dataclass
class PackedColumn:
    """A frame-of-reference + bit-packed int32 column (layout: agg_packed in agg.h).
    `blocks` and `payload` are numpy arrays (host) or torch tensors (device or pinned)."""
    blocks: object
    payload: object
    n: int
    payload_words: int

    def _ptr(self, x) -> int:
        if x is None:
            return 0
        return x.data_ptr() if hasattr(x, "data_ptr") else x.ctypes.data

    def struct(self) -> Packed:
        return Packed(self._ptr(self.blocks), self._ptr(self.payload), self.n, self.payload_words, I32, 0)

    @property
    def nbytes(self) -> int:
        return 16 * (-(-self.n // PACK_BLOCK)) + 4 * self.payload_words

    def to(self, where: str) -> "PackedColumn":
        """Copy to 'cuda' (device) or 'pinned' (page-locked host) torch tensors."""
        torch = _torch()
        np = _np()
        b = torch.from_numpy(np.ascontiguousarray(self.blocks).view(np.uint8).copy())
        p = torch.from_numpy(np.ascontiguousarray(self.payload).view(np.int32).copy())
        if where == "pinned":
            return PackedColumn(b.pin_memory(), p.pin_memory(), self.n, self.payload_words)
        return PackedColumn(b.to(where), p.to(where), self.n, self.payload_words)


def pack_i32(x, threads: int = 0) -> PackedColumn:
    """Encode an int32 column (numpy array or CPU tensor) on the host."""
    np = _np()
    if hasattr(x, "numpy"):
        x = x.numpy()
    x = np.ascontiguousarray(x, dtype=np.int32)
    n = x.size
    bound = ctypes.c_int64()
    _check(lib().agg_pack_bound(n, ctypes.byref(bound)), "agg_pack_bound")
    blocks = np.zeros(-(-n // PACK_BLOCK), dtype=block_dtype())
    payload = np.zeros(max(1, bound.value), dtype=np.uint32)
    used = ctypes.c_int64()
    _check(lib().agg_pack_i32(x.ctypes.data if n else None, n, blocks.ctypes.data if n else None,
                              payload.ctypes.data, payload.size, ctypes.byref(used), int(threads)),
           "agg_pack_i32")
    return PackedColumn(blocks, payload[:max(1, used.value)].copy(), n, used.value)
