"""Coupled ("p") algorithms, Fast Two-Sum renormalisation and chains in the
oracle (no GPU).

Pins, each independent of the code under test:

* Fast Two-Sum (Algorithm 1.1): s + t = a + b exactly whenever |a| >= |b|,
  checked in rational arithmetic.
* MPF1 drops x1 y1 from MTF1; on operands whose products and sums are all
  exact (small-integer mantissas) z1 must be e00 + x0 y1 + x1 y0 exactly,
  which a dropped or an extra term changes.  On coupled random operands
  |z1 - dz0| <= |x1 y1| + gamma_3 (|e00| + |x0 y1| + |x1 y0|).
* DPF1 divides by y0 only: on exact cases z1 = (x1 - z0 y1) / y0 exactly
  (DTF1 would divide by y0 + y1).  Derived bound, rho = y1 / y0, R1 = x1 - z0 y1:
  |z1 - dz0| <= |dz0| ((1 + |rho|)(1 + u)^2 - 1) + u (1 + u)^2 |R1| / |y0|.
* RPF1 is one Newton step for sqrt(u0 + u1) from v0 = sqrt(u0): with
  delta = S - v0 and rho = delta / (2 v0) the step gives delta (1 + rho)
  before its two roundings, so |z1 - delta| <= |delta| ((1 + |rho|)(1 + u)^2 - 1),
  S from mpmath at 400 bits.  On perfect squares z1 = x1 / (2 z0) exactly.
* The paper: with a dotted operand the coupled forms are literally the
  twofold ones (MPF1.1 = MTF1.1, DPF1.1 = DTF1.1).
* The paper's renormalisation example: adding 1 to a binary32 accumulator
  saturates at z0 = z1 = 2^24 without renormalising and stays exact with
  it (here 2^25 + 2^20 additions, and a run that ends exactly at 2^48).
* Chains of one step equal the single operations; the accumulator of the
  Applications section equals the twofold add chain.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from exact import F, U, bits_equal, gamma, rn, ulp
from test_oracle_eft import twofold

DTYPES = [np.float64, np.float32]
N = 1500


def coupled_operands(dtype, n, seed):
    """Coupled twofolds: |x1| < ulp(x0) / 2."""
    dtype = np.dtype(dtype)
    g = np.random.default_rng(seed)
    x0 = (g.uniform(1, 2, n) * np.where(g.integers(0, 2, n) == 1, -1, 1)
          * np.exp2(g.integers(-6, 7, n))).astype(dtype)
    x1 = (x0.astype(np.float64) * g.uniform(-0.5, 0.5, n) * float(U[dtype])).astype(dtype)
    return x0, x1


def small_int_operands(dtype, n, seed):
    """Twofolds whose parts are small integers times powers of two, far
    apart, so that every product and sum in MPF1 is exact."""
    g = np.random.default_rng(seed)
    sh = 20 if np.dtype(dtype) == np.float64 else 8

    def part(e):
        return (g.integers(-63, 64, n) * np.exp2(e)).astype(dtype)

    x0 = part(g.integers(-3, 4, n))
    y0 = part(g.integers(-3, 4, n))
    x1 = part(g.integers(-3, 4, n) - sh)
    y1 = part(g.integers(-3, 4, n) - sh)
    return x0, x1, y0, y1


# ---- Fast Two-Sum -----------------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_two_sum_is_exact_when_ordered(dtype):
    a, b = twofold(dtype, N, 41)
    swap = np.abs(a) < np.abs(b)
    a, b = np.where(swap, b, a).astype(dtype), np.where(swap, a, b).astype(dtype)
    s, t = oracle.fast_two_sum(a, b)
    for i in range(N):
        assert F(s[i]) + F(t[i]) == F(a[i]) + F(b[i]), i
        assert s[i] == rn(F(a[i]) + F(b[i]), dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_renorm_makes_coupled_output(dtype):
    z0, z1 = twofold(dtype, N, 43)  # |z1| up to 8 |z0|: the order is not given
    keep = np.abs(z0) >= np.abs(z1)
    s, t = oracle.renorm(z0, z1)
    for i in np.flatnonzero(keep):
        assert F(s[i]) + F(t[i]) == F(z0[i]) + F(z1[i])
        assert abs(F(t[i])) <= ulp(s[i], dtype) / 2


# ---- MPF1 ---------------------------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
def test_mpf1_exact_cases(dtype):
    x0, x1, y0, y1 = small_int_operands(dtype, N, 45)
    z0, z1 = oracle.coupled("mul", x0, x1, y0, y1)
    for i in range(N):
        assert z0[i] == x0[i] * y0[i]
        want = F(x0[i]) * F(y1[i]) + F(x1[i]) * F(y0[i])  # e00 = 0 here
        assert F(z1[i]) == want, i


@pytest.mark.parametrize("dtype", DTYPES)
def test_mpf1_bound_on_coupled_operands(dtype):
    x0, x1 = coupled_operands(dtype, N, 47)
    y0, y1 = coupled_operands(dtype, N, 48)
    z0, z1 = oracle.coupled("mul", x0, x1, y0, y1)
    for i in range(N):
        assert z0[i] == x0[i] * y0[i]
        e00 = F(x0[i]) * F(y0[i]) - F(z0[i])
        dz0 = (F(x0[i]) + F(x1[i])) * (F(y0[i]) + F(y1[i])) - F(z0[i])
        b = abs(F(x1[i]) * F(y1[i])) + gamma(3, dtype) * (
            abs(e00) + abs(F(x0[i]) * F(y1[i])) + abs(F(x1[i]) * F(y0[i])))
        assert abs(F(z1[i]) - dz0) <= b, i


# ---- DPF1 ---------------------------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
def test_dpf1_exact_cases(dtype):
    g = np.random.default_rng(49)
    n = N
    q = g.integers(-40, 41, n)
    q[q == 0] = 1
    k = g.integers(-4, 5, n)
    sh = 20 if np.dtype(dtype) == np.float64 else 8
    y0 = np.exp2(k).astype(dtype)
    x0 = (q * np.exp2(k)).astype(dtype)  # x0 / y0 = q exactly
    y1 = (g.integers(-63, 64, n) * np.exp2(k - sh)).astype(dtype)
    x1 = (g.integers(-63, 64, n) * np.exp2(k - sh)).astype(dtype)
    z0, z1 = oracle.coupled("div", x0, x1, y0, y1)
    for i in range(n):
        assert F(z0[i]) == q[i]
        want = (F(x1[i]) - F(z0[i]) * F(y1[i])) / F(y0[i])
        assert F(z1[i]) == want, i


@pytest.mark.parametrize("dtype", DTYPES)
def test_dpf1_dotted_dividend_exact_cases(dtype):
    """A dotted dividend over a coupled divisor is DPF1 with x1 = +0, so on
    exact cases z1 = -z0 y1 / y0 exactly (zero if y1 were dropped)."""
    g = np.random.default_rng(50)
    n = N
    q = g.integers(-40, 41, n)
    q[q == 0] = 1
    k = g.integers(-4, 5, n)
    sh = 20 if np.dtype(dtype) == np.float64 else 8
    y0 = np.exp2(k).astype(dtype)
    x0 = (q * np.exp2(k)).astype(dtype)
    y1 = (g.integers(-63, 64, n) * np.exp2(k - sh)).astype(dtype)
    y1[y1 == 0] = np.exp2(k[y1 == 0] - sh).astype(dtype)
    z0, z1 = oracle.coupled("div", x0, None, y0, y1)
    for i in range(n):
        assert F(z0[i]) == q[i]
        assert F(z1[i]) == -F(z0[i]) * F(y1[i]) / F(y0[i]), i


@pytest.mark.parametrize("dtype", DTYPES)
def test_dpf1_bound_on_coupled_operands(dtype):
    x0, x1 = coupled_operands(dtype, N, 51)
    y0, y1 = coupled_operands(dtype, N, 52)
    u = U[np.dtype(dtype)]
    z0, z1 = oracle.coupled("div", x0, x1, y0, y1)
    for i in range(N):
        assert z0[i] == x0[i] / y0[i]
        ys = F(y0[i]) + F(y1[i])
        dz0 = (F(x0[i]) + F(x1[i])) / ys - F(z0[i])
        rho = abs(F(y1[i]) / F(y0[i]))
        R1 = F(x1[i]) - F(z0[i]) * F(y1[i])
        b = abs(dz0) * ((1 + rho) * (1 + u) ** 2 - 1) + u * (1 + u) ** 2 * abs(R1) / abs(F(y0[i]))
        assert abs(F(z1[i]) - dz0) <= b, i


# ---- RPF1 ---------------------------------------------------------------------

def _mp(q: Fraction):
    return mpmath.mpf(q.numerator) / q.denominator


@pytest.mark.parametrize("dtype", DTYPES)
def test_rpf1_newton_bound(dtype):
    x0, x1 = coupled_operands(dtype, 600, 53)
    x0 = np.abs(x0)
    z0, z1 = oracle.coupled("sqrt", x0, x1)
    mpmath.mp.prec = 400
    u = _mp(U[np.dtype(dtype)])
    for i in range(x0.size):
        assert z0[i] == np.sqrt(x0[i])
        S = mpmath.sqrt(_mp(F(x0[i]) + F(x1[i])))
        delta = S - mpmath.mpf(float(z0[i]))
        rho = abs(delta) / (2 * mpmath.mpf(float(z0[i])))
        b = abs(delta) * ((1 + rho) * (1 + u) ** 2 - 1)
        assert abs(mpmath.mpf(float(z1[i])) - delta) <= b, i


@pytest.mark.parametrize("dtype", DTYPES)
def test_rpf1_exact_on_perfect_squares(dtype):
    g = np.random.default_rng(55)
    q = g.integers(1, 2000, 500)
    k = g.integers(-3, 4, 500)
    z = (q * np.exp2(k)).astype(dtype)
    x0 = (z.astype(np.float64) ** 2).astype(dtype)  # exact: q < 2^11
    x1 = (g.integers(-63, 64, 500) * np.exp2(2 * k - 30)).astype(dtype)
    z0, z1 = oracle.coupled("sqrt", x0, x1)
    for i in range(500):
        assert z0[i] == z[i]
        assert F(z1[i]) == rn(F(x1[i]) / (2 * F(z0[i])), dtype), i


# ---- dotted forms -----------------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_dotted_coupled_forms_are_the_twofold_ones(op, dtype):
    x0, x1 = twofold(dtype, N, 57)
    y0, y1 = twofold(dtype, N, 58)
    f = getattr(oracle, op)
    for args in ((x0, x1, y0, None), (x0, None, y0, None)):
        assert bits_equal(oracle.coupled(op, *args)[1], f(*args)[1]).all()
    if op in ("add", "sub"):  # no coupled algorithm of their own
        assert bits_equal(oracle.coupled(op, x0, x1, y0, y1)[1], f(x0, x1, y0, y1)[1]).all()
        assert bits_equal(oracle.coupled(op, x0, None, y0, y1)[1], f(x0, None, y0, y1)[1]).all()
    assert bits_equal(oracle.coupled("sqrt", np.abs(x0), None)[1], oracle.sqrt(np.abs(x0), None)[1]).all()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div", "sqrt"])
def test_dekker_mode_is_coupled_then_fast_two_sum(op, dtype):
    x0, x1 = coupled_operands(dtype, N, 59)
    y0, y1 = coupled_operands(dtype, N, 60)
    if op == "sqrt":
        x0 = np.abs(x0)
    a = oracle.coupled(op, x0, x1, y0, y1)
    b = oracle.coupled(op, x0, x1, y0, y1, renorm=True)
    for i in range(N):
        if abs(a[0][i]) >= abs(a[1][i]):
            assert F(b[0][i]) + F(b[1][i]) == F(a[0][i]) + F(a[1][i])
            assert abs(F(b[1][i])) <= ulp(b[0][i], dtype) / 2


# ---- the paper's renormalisation example ----------------------------------

def test_counting_ones_saturates_without_renormalising():
    f32 = np.float32
    steps = 2 ** 25 + 2 ** 20
    one = np.ones(1, f32)
    z0, z1 = oracle.chain("add", "twofold", steps, np.zeros(1, f32), None, one, None)
    assert (z0[0], z1[0]) == (2.0 ** 24, 2.0 ** 24)
    z0, z1 = oracle.chain("add", "dekker", steps, np.zeros(1, f32), None, one, None)
    assert (F(z0[0]), F(z1[0])) == (steps, 0)


def test_counting_ones_reaches_2_48_with_renormalising():
    f32 = np.float32
    z0, z1 = oracle.chain("add", "dekker", 2 ** 20, np.array([2.0 ** 48], f32), np.array([-(2.0 ** 20)], f32),
                          np.ones(1, f32), None)
    assert (F(z0[0]), F(z1[0])) == (2 ** 48, 0)


# ---- chains -------------------------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div", "sqrt"])
def test_one_step_chain_is_the_operation(op, dtype):
    x0, x1 = twofold(dtype, N, 61)
    y0, y1 = twofold(dtype, N, 62)
    if op == "sqrt":
        x0, x1 = np.abs(x0), np.abs(x1)
    single = {"sqrt": lambda: oracle.sqrt(x0, x1)}.get(op, lambda: getattr(oracle, op)(x0, x1, y0, y1))()
    got = oracle.chain(op, "twofold", 1, x0, x1, y0, y1)
    assert bits_equal(got[0], single[0]).all() and bits_equal(got[1], single[1]).all()
    if op != "sqrt":
        single = getattr(oracle, op)(x0, x1, y0, None)
        got = oracle.chain(op, "twofold", 1, x0, x1, y0, None)
        assert bits_equal(got[1], single[1]).all()
    for mode, renorm in (("coupled", False), ("dekker", True)):
        single = oracle.coupled(op, x0, x1, y0, y1, renorm=renorm)
        got = oracle.chain(op, mode, 1, x0, x1, y0, y1)
        assert bits_equal(got[0], single[0]).all() and bits_equal(got[1], single[1]).all()
    plain = oracle.plain_chain(op, 1, x0, y0)
    want = oracle.plain(op, x0) if op == "sqrt" else oracle.plain(op, x0, y0)
    assert bits_equal(plain, want).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_zero_step_chain_is_the_start_value(dtype):
    x0, x1 = twofold(dtype, 100, 63)
    z = oracle.chain("mul", "twofold", 0, x0, x1, x0, x1)
    assert bits_equal(z[0], x0).all() and bits_equal(z[1], x1).all()
    z = oracle.chain("mul", "twofold", 0, x0, None, x0, x1)
    assert bits_equal(z[0], x0).all() and (z[1] == 0).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_add_chain_is_the_clock_accumulator(dtype):
    t0, t1 = np.asarray([0.1], dtype), np.asarray([np.float64(0.1) - np.float64(dtype(0.1))], dtype)
    z = oracle.chain("add", "twofold", 360000, np.zeros(1, dtype), np.zeros(1, dtype), t0, t1)
    s = oracle.accumulate(360000, t0[0], t1[0])
    assert bits_equal(z[0], [s[0]]).all() and bits_equal(z[1], [s[1]]).all()
