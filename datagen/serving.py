"""Seeded serving workloads (request streams), inputs only.

A stream of aggregation requests with Poisson arrivals (exponential gaps),
column lengths log-uniform in [n_min, n_max], uniformly drawn functions, and a
resident / shipped split: a resident request reads a slice of a "hot" region
preloaded in HBM, a shipped request reads a slice of a host arena that must be
copied over PCIe.  With `repeat_frac` > 0 some shipped requests repeat an
earlier shipped column (same slice, same column id), so a resident cache can
serve them.  Nothing here aggregates anything.
"""
from __future__ import annotations

import math

import numpy as np

OPS = ["sum", "min", "max", "count", "avg"]


def request_stream(nreq: int, seed: int, n_min: int, n_max: int, rate_per_s: float,
                   resident_frac: float = 0.3, hot_items: int = 0, arena_items: int = 0,
                   repeat_frac: float = 0.0, ops=OPS) -> list:
    """Request specs: dicts with n, arrival_s, op, resident, offset (items into
    the hot region or the host arena) and column_id."""
    r = np.random.default_rng(seed)
    t = 0.0
    out = []
    shipped = []
    for i in range(nreq):
        t += r.exponential(1.0 / rate_per_s)
        op = ops[int(r.integers(0, len(ops)))]
        resident = bool(r.random() < resident_frac)
        if not resident and shipped and r.random() < repeat_frac:
            prev = shipped[int(r.integers(0, len(shipped)))]
            out.append(dict(n=prev["n"], arrival_s=t, op=op, resident=False, offset=prev["offset"],
                            column_id=prev["column_id"]))
            continue
        n = int(math.exp(r.uniform(math.log(n_min), math.log(n_max))))
        space = hot_items if resident else arena_items
        n = min(n, space)
        offset = int(r.integers(0, space - n + 1))
        req = dict(n=n, arrival_s=t, op=op, resident=resident, offset=offset,
                   column_id=(i + (1 << 40)) if not resident else -(i + 1))
        out.append(req)
        if not resident:
            shipped.append(req)
    return out


def mean_bytes(n_min: int, n_max: int, width: int) -> float:
    """Mean bytes of a log-uniform length in [n_min, n_max]."""
    return width * (n_max - n_min) / math.log(n_max / n_min)
