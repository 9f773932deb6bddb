"""The group-by float-sum rounding (csrc/agg_digits.hpp), compiled for the host.

The GPU keeps each float group sum exactly as base-2^32 fixed-point digits and
rounds it once to double.  This checks that rounding against Python's exact
rational arithmetic (int / int true division is correctly rounded, ties to
even) on random digit vectors, exact halfway cases and the non-finite flags."""
import ctypes
import math
import os
import random
import subprocess
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_10030_amd", "csrc")
NDIG = 9


@pytest.fixture(scope="module")
def d2d(tmp_path_factory):
    d = tmp_path_factory.mktemp("digits")
    src = d / "h.cpp"
    src.write_text('#define __host__\n#define __device__\n#include "agg_digits.hpp"\n'
                   'extern "C" double d2d(const int64_t* s, int f) { return agg::gb::digits_to_double(s, f); }\n')
    lib = d / "h.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wno-unknown-pragmas", "-fPIC", "-shared",
                           "-I", CSRC, str(src), "-o", str(lib)])
    L = ctypes.CDLL(str(lib))
    L.d2d.restype = ctypes.c_double
    L.d2d.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    return lambda ds, f=0: L.d2d((ctypes.c_int64 * NDIG)(*ds), f)


def exact(ds):
    num = sum(x << (32 * k) for k, x in enumerate(ds))
    return num / (1 << 149)          # int / int: correctly rounded


def test_random_digit_vectors(d2d):
    r = random.Random(7)
    for trial in range(30000):
        mode = trial % 4
        ds = []
        for k in range(NDIG):
            if mode == 0:
                ds.append(r.randint(-2**40, 2**40))
            elif mode == 1:
                ds.append(r.choice([0, 0, 0, r.randint(-2**62, 2**62)]))
            elif mode == 2:
                ds.append(r.choice([0, 1, -1, 2**31, 2**32 - 1, -(2**32), r.randint(-3, 3)]))
            else:
                ds.append(r.getrandbits(32) if k < NDIG - 1 else r.randint(0, 2**20))
        assert d2d(ds) == exact(ds), ds


def test_halfway_cases_round_to_even(d2d):
    for e in range(-148, 150, 3):
        for m in (2**52, 2**52 + 1, 2**53 - 1, 2**52 + 12345):
            fx = (2 * m + 1) << (e - 1 + 149)     # exactly between two doubles
            if fx >> (32 * NDIG):
                continue
            ds = [(fx >> (32 * k)) & 0xFFFFFFFF for k in range(NDIG)]
            want = exact(ds)
            assert d2d(ds) == want
            assert d2d([-x for x in ds]) == -want
            up = list(ds)
            up[0] += 1                             # just above the tie: rounds up
            assert d2d(up) == exact(up)


def test_zero_small_and_flags(d2d):
    z = [0] * NDIG
    assert d2d(z) == 0.0
    assert d2d([1] + [0] * (NDIG - 1)) == 2.0**-149
    assert d2d([-3] + [0] * (NDIG - 1)) == -3 * 2.0**-149
    assert math.isnan(d2d(z, 1)) and math.isnan(d2d(z, 2 | 4)) and math.isnan(d2d(z, 1 | 2))
    assert d2d(z, 2) == math.inf and d2d(z, 4) == -math.inf


def test_float_sums_as_the_gpu_accumulates_them(d2d):
    """Digits built the way the kernel adds a float (two digits per float: the
    signed product split as lo + hi * 2^32 with 0 <= lo < 2^32), and built with
    each digit negated instead (digits of either sign): both round to the exact
    sum."""
    import numpy as np
    r = random.Random(3)
    for _ in range(300):
        xs = (np.array([r.gauss(0, 1) for _ in range(50)]) *
              np.exp2(np.array([r.randint(-140, 120) for _ in range(50)]))).astype(np.float32)
        xs = xs[np.isfinite(xs)]
        ds = [0] * NDIG
        dn = [0] * NDIG
        for x in xs.tolist():
            # |x| = mm * 2^(kk - 149): mantissa and exponent from the float's bits
            bits = int(np.float32(abs(x)).view(np.uint32))
            biased, frac = bits >> 23, bits & 0x7FFFFF
            mm = (frac | 0x800000) if biased else frac
            kk = biased - 1 if biased else 0
            v = mm << (kk & 31)
            sv = -v if x < 0 else v
            ds[kk >> 5] += sv & 0xFFFFFFFF
            ds[(kk >> 5) + 1] += sv >> 32
            lo, hi = v & 0xFFFFFFFF, v >> 32
            if x < 0:
                lo, hi = -lo, -hi
            dn[kk >> 5] += lo
            dn[(kk >> 5) + 1] += hi
        want = float(sum((Fraction(float(x)) for x in xs.tolist()), Fraction(0)))
        assert d2d(ds) == want
        assert d2d(dn) == want
