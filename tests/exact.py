"""Exact rational arithmetic helpers for the tests.

Every value here is an exact ``fractions.Fraction``; rounding to binary64 or
binary32 is done by ``rn`` from first principles (round to nearest, ties to
even, with gradual underflow and overflow to infinity), so the checks built
on it do not depend on the code under test.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

# (precision p, minimum normal exponent, maximum exponent) of each format
FORMATS = {
    np.dtype(np.float64): (53, -1022, 1023),
    np.dtype(np.float32): (24, -126, 127),
}
U = {np.dtype(np.float64): Fraction(1, 2 ** 53), np.dtype(np.float32): Fraction(1, 2 ** 24)}


def F(x) -> Fraction:
    """Exact value of a finite binary64 / binary32 number."""
    return Fraction(float(x))


def _ilog2(q: Fraction) -> int:
    """floor(log2(q)) for q > 0, exactly."""
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1
    elif Fraction(2) ** (e + 1) <= q:
        e += 1
    return e


def rn(q: Fraction, dtype=np.float64):
    """q rounded to nearest-even in the given format (numpy scalar)."""
    dtype = np.dtype(dtype)
    p, emin, emax = FORMATS[dtype]
    if q == 0:
        return dtype.type(0.0)
    neg = q < 0
    a = -q if neg else q
    e = max(_ilog2(a), emin)
    quantum = Fraction(2) ** (e - p + 1)
    m = a / quantum
    k = m.numerator // m.denominator
    r = m - k
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and k % 2 == 1):
        k += 1
    v = k * quantum
    if v >= Fraction(2) ** (emax + 1):
        out = np.inf
    else:
        out = float(v)  # exact: v has at most p significant bits
    out = -out if neg else out
    return dtype.type(out)


def ulp(x, dtype=np.float64) -> Fraction:
    """Unit in the last place of a finite nonzero x (spacing above |x|)."""
    dtype = np.dtype(dtype)
    p, emin, _ = FORMATS[dtype]
    a = abs(F(x))
    if a == 0:
        return Fraction(2) ** (emin - p + 1)
    e = max(_ilog2(a), emin)
    return Fraction(2) ** (e - p + 1)


def gamma(k: int, dtype=np.float64) -> Fraction:
    """Higham's gamma_k = k u / (1 - k u)."""
    u = U[np.dtype(dtype)]
    return k * u / (1 - k * u)


def same(a, b) -> bool:
    """Bitwise equality of two numbers, any NaN equal to any NaN."""
    a = np.asarray(a)
    b = np.asarray(b)
    if np.isnan(a) and np.isnan(b):
        return True
    return a.tobytes() == b.tobytes()


def bits_equal(a, b) -> np.ndarray:
    """Elementwise bit equality of two arrays (NaN matches any NaN)."""
    a = np.asarray(a)
    b = np.asarray(b)
    ui = np.uint64 if a.dtype == np.float64 else np.uint32
    eq = a.view(ui) == b.view(ui)
    return eq | (np.isnan(a) & np.isnan(b))
