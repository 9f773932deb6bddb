"""A step-by-step numpy model of the float32 SUM's canonical reduction shape.

Test infrastructure only.  It is not the oracle (the oracle is the exact sum,
`oracle/`); it restates, in numpy float32 / float64 arithmetic (IEEE
round-to-nearest, no fused operations), the order of operations that
`include/agg.h` documents for a float32 column:

* the column's bytes are cut into segments of S bytes (agg_canonical_shape);
* in a segment, lane l folds the 16-byte vectors at r * 1024 + 16 l,
  r = 0, 1, ..., each of the 4 components into its own accumulator; a
  partial last round gives a lane its whole vector or its first items;
* compensated mode: Neumaier's update per item, an exact two-sum
  renormalisation of every accumulator after each block of 8 rounds and once
  after the last round, components merged as (c0 + c1) + (c2 + c3), the 64
  lanes merged as a balanced tree in lane order (the butterfly's merges are
  symmetric, so lane 0's value is that tree), segment partial s + c in double;
* plain / f64-combine modes: float32 additions, the same trees, the segment
  total kept in float32 or widened to double;
* the nseg partials: lane L of 256 folds L, L + 256, ... in order from zero,
  each 64-lane wave merges as a balanced tree, then (w0 + w1) + (w2 + w3).

It serves two purposes: on the CPU, exercising the error-bound derivation of
`aggcheck.py` on inputs built to make rounding errors add up; on the GPU,
checking that the kernels follow the documented shape bit for bit.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
F64 = np.float64
RENORM_ROUNDS = 8
ROUND_ITEMS = 256          # 64 lanes x 4 float32 items per 1 KiB round


def seg_bytes_for(n: int, width: int = 4) -> int:
    total = n * width
    seg = 16 * 1024
    target = -(-total // 8192)
    while seg < target:
        seg <<= 1
    return seg


# ------------------------------------------------------------ float32 steps
def two_sum(a, b):
    """Knuth's two-sum in float32: t = fl(a + b), e = a + b - t exactly."""
    t = (a + b).astype(F32)
    bb = (t - a).astype(F32)
    e = ((a - (t - bb)).astype(F32) + (b - bb).astype(F32)).astype(F32)
    return t, e


def neumaier_add(s, c, x, mask=None):
    t = (s + x).astype(F32)
    s_big = np.abs(s) >= np.abs(x)
    big = np.where(s_big, s, x)
    small = np.where(s_big, x, s)
    c2 = (c + ((big - t).astype(F32) + small).astype(F32)).astype(F32)
    if mask is None:
        return t, c2
    return np.where(mask, t, s), np.where(mask, c2, c)


def neu_merge(a, b):
    (sa, ca), (sb, cb) = a, b
    t, e = two_sum(sa, sb)
    return two_sum(t, ((ca + cb).astype(F32) + e).astype(F32))


def tree(vals, merge, axis):
    """Balanced pairwise tree over `axis` (length a power of two), adjacent
    pairs first.  vals is an array or a tuple of arrays (a pair per element)."""
    is_t = isinstance(vals, tuple)

    def take(v, start):
        return np.take(v, np.arange(start, v.shape[axis], 2), axis=axis)

    while (vals[0] if is_t else vals).shape[axis] > 1:
        if is_t:
            vals = merge(tuple(take(v, 0) for v in vals), tuple(take(v, 1) for v in vals))
        else:
            vals = merge(take(vals, 0), take(vals, 1))
    if is_t:
        return tuple(np.squeeze(v, axis=axis) for v in vals)
    return np.squeeze(vals, axis=axis)


# ------------------------------------------------------------ lane folds
def lane_fold_neumaier(rounds, mask=None, renorm=RENORM_ROUNDS, full=None):
    """Fold rounds[r, ...] (float32) into Neumaier pairs, round r in order.
    mask[r, ...] (optional) marks the items present; `full` is the number of
    complete rounds (default: all), after which a partial round may follow.
    A block renormalisation follows each complete round r with
    (r + 1) % renorm == 0, and one more closes the fold.  renorm = 0 disables
    both (the variant whose correction term is never renormalised)."""
    full = rounds.shape[0] if full is None else full
    s = np.zeros(rounds.shape[1:], F32)
    c = np.zeros(rounds.shape[1:], F32)
    for r in range(rounds.shape[0]):
        s, c = neumaier_add(s, c, rounds[r], None if mask is None else mask[r])
        if renorm and r < full and (r + 1) % renorm == 0:
            s, c = two_sum(s, c)
    if renorm:
        s, c = two_sum(s, c)
    return s, c


def lane_fold_plain(rounds, mask=None):
    a = np.zeros(rounds.shape[1:], F32)
    for r in range(rounds.shape[0]):
        b = (a + rounds[r]).astype(F32)
        a = b if mask is None else np.where(mask[r], b, a)
    return a


# ------------------------------------------------------------ segments
def _segment_rounds(xseg_items: np.ndarray):
    """(rounds, mask) of shape (R, 64, 4) for one segment's items, the
    partial last round masked."""
    nitems = xseg_items.size
    nr = -(-nitems // ROUND_ITEMS)
    pad = np.zeros(nr * ROUND_ITEMS, F32)
    pad[:nitems] = xseg_items
    mask = np.zeros(nr * ROUND_ITEMS, bool)
    mask[:nitems] = True
    return pad.reshape(nr, 64, 4), mask.reshape(nr, 64, 4)


def segment_partials(x: np.ndarray, prec: str, renorm: int = RENORM_ROUNDS) -> np.ndarray:
    """The segment partials of the float32 column x in precision mode prec
    ('neumaier', 'f32' or 'f64_combine'): float64 except plain float32."""
    x = np.ascontiguousarray(x, F32)
    n = x.size
    if n == 0:
        return np.zeros(0, F64)
    seg_items = seg_bytes_for(n) // 4
    nseg = -(-n // seg_items)
    nfull = n // seg_items
    parts = []
    groups = []
    if nfull:
        rounds = x[: nfull * seg_items].reshape(nfull, seg_items // ROUND_ITEMS, 64, 4).transpose(1, 0, 2, 3)
        groups.append((rounds, None, rounds.shape[0]))
    if nseg > nfull:
        tail = x[nfull * seg_items:]
        r, m = _segment_rounds(tail)
        groups.append((r[:, None], m[:, None], tail.size // ROUND_ITEMS))
    for rounds, mask, full in groups:
        if prec == "neumaier":
            s, c = lane_fold_neumaier(rounds, mask, renorm, full)
            a = (s, c)
            comp = neu_merge(neu_merge((a[0][..., 0], a[1][..., 0]), (a[0][..., 1], a[1][..., 1])),
                             neu_merge((a[0][..., 2], a[1][..., 2]), (a[0][..., 3], a[1][..., 3])))
            ws, wc = tree(comp, neu_merge, axis=1)
            parts.append(ws.astype(F64) + wc.astype(F64))
        else:
            a = lane_fold_plain(rounds, mask)
            comp = ((a[..., 0] + a[..., 1]).astype(F32) + (a[..., 2] + a[..., 3]).astype(F32)).astype(F32)
            w = tree(comp, lambda p, q: (p + q).astype(F32), axis=1)
            parts.append(w.astype(F64) if prec == "f64_combine" else w.astype(F32))
    return np.concatenate(parts)


def combine(parts: np.ndarray) -> float:
    """The canonical merge of the segment partials (in their own precision)."""
    dt = parts.dtype.type
    nseg = parts.size
    lanes = np.zeros(256, dt)
    for k0 in range(0, nseg, 256):
        chunk = parts[k0:k0 + 256]
        lanes[: chunk.size] = (lanes[: chunk.size] + chunk).astype(dt)
    waves = tree(lanes.reshape(4, 64), lambda p, q: (p + q).astype(dt), axis=1)
    total = ((waves[0] + waves[1]).astype(dt) + (waves[2] + waves[3]).astype(dt)).astype(dt)
    return float(total)


def model_sum(x: np.ndarray, prec: str, renorm: int = RENORM_ROUNDS) -> float:
    """The float32 column's SUM as the canonical shape computes it (a double)."""
    return combine(segment_partials(x, prec, renorm))
