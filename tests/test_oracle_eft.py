"""The oracle's error-free transforms and strict variants, pinned by exact
rational arithmetic (no GPU).

Pins (Background section, exact transforms and Algorithms 1.2, 2.2, 3, 4,
5; Algorithms ATF1.1, STF1.1, DTF1.1.1, RPF1.1 of the Algorithms section):
  * a + b = s + t, a - b = d + t, a b = p + e, a = q b + r, a = c^2 + d hold
    exactly, with s, d, p, q, c the correctly rounded results, on small-
    exponent operands where nothing underflows;
  * the *.1 add/sub variants are strict: z1 = RN(dz0) exactly;
  * dividing dotted numbers (DTF1.1.1) gives z1 = RN(dz0), |z1| <= ulp(z0)/2;
  * the dotted square root (RPF1.1) is coupled, |z1| <= ulp(z0)/2, and within
    its derived bound of the true deviation;
  * z0 of every operation equals numpy's own IEEE operation.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from exact import F, U, bits_equal, rn, ulp

DTYPES = [np.float64, np.float32]


def small_cases(dtype, n=1000, seed=11):
    """Operands with full random mantissas and exponents in [-8, 8], plus
    ties, exact sums, a = -b and powers of two (nothing underflows)."""
    dtype = np.dtype(dtype)
    g = np.random.default_rng(seed)
    p = 53 if dtype == np.float64 else 24
    def draw(m):
        mant = 1 + g.integers(0, 2 ** (p - 1), m).astype(np.float64) / 2 ** (p - 1)
        sign = np.where(g.integers(0, 2, m) == 1, -1.0, 1.0)
        return (sign * np.ldexp(mant, g.integers(-8, 9, m))).astype(dtype)
    a, b = draw(n), draw(n)
    special_a = np.array([1.0, 1.0, 3.0, 2.0 ** 7, -5.0, 1.5, 1.0, 0.75], dtype)
    special_b = np.array([2.0 ** -p, -1.0, -3.0, 2.0 ** -3, 5.0, 2.0 ** (1 - p), 3.0, 0.25], dtype)
    return np.concatenate([a, special_a]), np.concatenate([b, special_b])


@pytest.mark.parametrize("dtype", DTYPES)
def test_two_sum_is_exact(dtype):
    a, b = small_cases(dtype)
    s, t = oracle.two_sum(a, b)
    for ai, bi, si, ti in zip(a, b, s, t):
        assert si == rn(F(ai) + F(bi), dtype)
        assert F(si) + F(ti) == F(ai) + F(bi)


@pytest.mark.parametrize("dtype", DTYPES)
def test_two_diff_is_exact(dtype):
    # Also pins the orientation of the lost parts: with the operands of
    # Algorithm 2.2's last two subtractions as printed, d + t = a - b fails
    # whenever the subtraction rounds (t comes out negated).
    a, b = small_cases(dtype)
    d, t = oracle.two_diff(a, b)
    rounded = 0
    for ai, bi, di, ti in zip(a, b, d, t):
        assert di == rn(F(ai) - F(bi), dtype)
        assert F(di) + F(ti) == F(ai) - F(bi)
        rounded += ti != 0
    assert rounded > 500


@pytest.mark.parametrize("dtype", DTYPES)
def test_two_prod_is_exact(dtype):
    a, b = small_cases(dtype)
    p, e = oracle.two_prod(a, b)
    for ai, bi, pi, ei in zip(a, b, p, e):
        assert pi == rn(F(ai) * F(bi), dtype)
        assert F(pi) + F(ei) == F(ai) * F(bi)


@pytest.mark.parametrize("dtype", DTYPES)
def test_division_remainder_is_exact(dtype):
    a, b = small_cases(dtype)
    q, r = oracle.div_rem(a, b)
    for ai, bi, qi, ri in zip(a, b, q, r):
        assert qi == rn(F(ai) / F(bi), dtype)
        assert F(qi) * F(bi) + F(ri) == F(ai)


@pytest.mark.parametrize("dtype", DTYPES)
def test_sqrt_residual_is_exact(dtype):
    a, _ = small_cases(dtype)
    a = np.abs(a)
    c, d = oracle.sqrt_rem(a)
    for ai, ci, di in zip(a, c, d):
        # c is the correctly rounded root: a lies strictly between the squares
        # of the midpoints to c's neighbours (a root is never a midpoint)
        lo = (F(ci) + F(np.nextafter(ci, dtype(-np.inf)))) / 2
        hi = (F(ci) + F(np.nextafter(ci, dtype(np.inf)))) / 2
        assert lo * lo < F(ai) < hi * hi
        assert F(ci) * F(ci) + F(di) == F(ai)


def twofold(dtype, n, seed, spread=True):
    """Twofold operands of mixed balance: coupled (|x1| ~ u|x0|), loose
    (|x1| ~ 2^-10 |x0|), comparable parts and inverse pairs."""
    dtype = np.dtype(dtype)
    g = np.random.default_rng(seed)
    x0 = (g.uniform(1, 2, n) * np.where(g.integers(0, 2, n) == 1, -1, 1)
          * np.exp2(g.integers(-6, 7, n))).astype(dtype)
    if not spread:
        scale = np.full(n, float(U[dtype]))
    else:
        scale = np.choose(g.integers(0, 4, n), [float(U[dtype]), 2.0 ** -10, 0.5, 8.0])
    x1 = (x0.astype(np.float64) * g.uniform(-1, 1, n) * scale).astype(dtype)
    return x0, x1


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["add", "sub"])
def test_add_sub_with_dotted_operand_is_strict(dtype, op):
    """ATF1.1 / STF1.1 (and the exchanged-operand forms) give z1 = RN(dz0)."""
    x0, x1 = twofold(dtype, 600, 3)
    y0, y1 = twofold(dtype, 600, 4)
    sign = 1 if op == "add" else -1
    f = getattr(oracle, op)
    z0, z1 = f(x0, x1, y0, None)              # twofold x, dotted y
    for i in range(x0.size):
        exact = F(x0[i]) + F(x1[i]) + sign * F(y0[i])
        assert z1[i] == rn(exact - F(z0[i]), dtype)
    z0, z1 = f(x0, None, y0, y1)              # dotted x, twofold y
    for i in range(x0.size):
        exact = F(x0[i]) + sign * (F(y0[i]) + F(y1[i]))
        assert z1[i] == rn(exact - F(z0[i]), dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["add", "sub", "mul"])
def test_dotted_operands_give_exact_transforms(dtype, op):
    a, b = small_cases(dtype)
    z0, z1 = getattr(oracle, op)(a, None, b, None)
    for ai, bi, s, t in zip(a, b, z0, z1):
        exact = {"add": F(ai) + F(bi), "sub": F(ai) - F(bi), "mul": F(ai) * F(bi)}[op]
        assert F(s) + F(t) == exact


@pytest.mark.parametrize("dtype", DTYPES)
def test_dotted_division_is_strict_and_coupled(dtype):
    a, b = small_cases(dtype)
    z0, z1 = oracle.div(a, None, b, None)
    for ai, bi, q0, q1 in zip(a, b, z0, z1):
        dz0 = F(ai) / F(bi) - F(q0)
        assert q1 == rn(dz0, dtype)
        assert abs(F(q1)) <= ulp(q0, dtype) / 2


@pytest.mark.parametrize("dtype", DTYPES)
def test_dotted_sqrt_is_coupled_and_accurate(dtype):
    """RPF1.1: z1 = (x0 - z0^2) / (2 z0) with the residual exact.  The true
    deviation is dz0 = h / (sqrt(x0) + z0); replacing sqrt(x0) + z0 by 2 z0
    changes it by the relative amount dz0 / (2 z0) <= u/2, and the division
    rounds once more: |z1 - dz0| <= (3u/2)(1 + u) |dz0|."""
    a, _ = small_cases(dtype)
    a = np.abs(a)
    z0, z1 = oracle.sqrt(a, None)
    u = U[np.dtype(dtype)]
    mpmath.mp.prec = 400
    for ai, c0, c1 in zip(a, z0, z1):
        assert abs(F(c1)) <= ulp(c0, dtype) / 2
        s = mpmath.sqrt(mpmath.mpf(float(ai)))
        dz0 = s - mpmath.mpf(float(c0))
        bound = mpmath.mpf(float(Fraction(3, 2) * u * (1 + u))) * abs(dz0)
        assert abs(mpmath.mpf(float(c1)) - dz0) <= bound


@pytest.mark.parametrize("dtype", DTYPES)
def test_z0_is_the_standard_result(dtype):
    """z0 of every operation is bitwise numpy's own IEEE operation."""
    x0, x1 = twofold(dtype, 4000, 5)
    y0, y1 = twofold(dtype, 4000, 6)
    for op, ref in (("add", np.add), ("sub", np.subtract), ("mul", np.multiply),
                    ("div", np.divide)):
        f = getattr(oracle, op)
        for xx1, yy1 in ((x1, y1), (x1, None), (None, y1), (None, None)):
            z0, _ = f(x0, xx1, y0, yy1)
            assert bits_equal(z0, ref(x0, y0)).all(), op
            assert bits_equal(oracle.plain(op, x0, y0), ref(x0, y0)).all(), op
    for xx1 in (np.abs(x1), None):
        z0, _ = oracle.sqrt(np.abs(x0), xx1)
        assert bits_equal(z0, np.sqrt(np.abs(x0))).all()
    assert bits_equal(oracle.plain("sqrt", np.abs(x0)), np.sqrt(np.abs(x0))).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_special_values_propagate(dtype):
    """No special-case handling: NaN and infinities flow through the basic
    operations (Algorithms section, methodic rules; DTF1.1.1 and RPF1 notes)."""
    t = np.dtype(dtype).type
    inf, nan = t(np.inf), t(np.nan)
    z0, z1 = oracle.div(np.array([1, 0, nan], dtype), None, np.array([0, 0, 1], dtype), None)
    assert z0[0] == inf and np.isnan(z1[0])          # y0 = 0: z0 infinite, z1 NaN
    assert np.isnan(z0[1]) and np.isnan(z1[1])       # 0/0
    assert np.isnan(z0[2]) and np.isnan(z1[2])       # NaN propagates
    z0, z1 = oracle.sqrt(np.array([-1, 0], dtype), None)
    assert np.isnan(z0[0]) and np.isnan(z1[0])       # negative argument: domain error
    assert z0[1] == 0 and np.isnan(z1[1])            # sqrt(0): 0/0 in z1 (reading)
    z0, z1 = oracle.add(np.array([inf], dtype), np.array([0], dtype),
                        np.array([1], dtype), np.array([0], dtype))
    assert z0[0] == inf and np.isnan(z1[0])          # inf - inf inside Two-Sum
