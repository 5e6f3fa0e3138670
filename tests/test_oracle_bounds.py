"""The general twofold operations against the exact deviation (no GPU).

For general (possibly overlapping) twofolds the paper promises no relative
accuracy, only that z1 approximates dz0 = z - z0.  Each test below checks
z1 against the exact dz0 (rational arithmetic, or mpmath at 400 bits for
square roots) within a bound derived from the operation's own rounding
steps, with u the unit roundoff and gamma_k = k u / (1 - k u):

  ATF1 / STF1: dz0 = x1 +- y1 + e, e = err(x0 +- y0) exact; two roundings:
      |z1 - dz0| <= gamma_2 (|x1| + |y1| + |e|)
  MTF1: dz0 = e00 + x0 y1 + x1 y0 + x1 y1 exactly; each term meets at most
      three roundings: |z1 - dz0| <= gamma_3 (|e00| + |x0y1| + |x1y0| + |x1y1|)
  MTF1.1: |z1 - dz0| <= gamma_2 (|e00| + |x1 y0|)
  DTF1: dz0 = (r0 + (x1 - z0 y1)) / (y0 + y1) with r0 exact; r1, c0, d0 and
      z1 each round once: |z1 - dz0| <= gamma_3 |dz0| + gamma_2 |x1 - z0 y1| / |y0 + y1|
  DTF1.1: |z1 - dz0| <= gamma_2 |dz0|
  RTF1: with S = sqrt(x0 + x1), u0 = RN(x0 + x1), v0 = RN(sqrt(u0)),
      delta = S - v0 and rho = |delta| / (2 v0), the Newton step is off by
      E = |delta| (1 + rho)(gamma_2 + rho / (1 - rho)), and the final
      Two-Diff / two additions give
      |z1 - dz0| <= E (1 + u) + u (1 + u)(|delta| + E + u |v0 - z0|) + u |dz0|

The operands mix the paper's balance classes (coupled, loose, comparable
parts, inverse pairs), so a dropped term, a wrong sign or an exchanged
operand in any step leaves one of these bounds violated.

FP32 twofolds are also judged against dz0 computed by the FP64 oracle on the
widened inputs (the paper's suggested way of checking float results), with
the same bounds at u = 2^-24 plus a slack for the reference's own error,
which is the same bound at u = 2^-53.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from exact import F, U, gamma, rn
from test_oracle_eft import twofold

DTYPES = [np.float64, np.float32]
N = 2000


def _cases(dtype, seed):
    x0, x1 = twofold(dtype, N, seed)
    y0, y1 = twofold(dtype, N, seed + 100)
    return x0, x1, y0, y1


def bound_add(x0, x1, y0, y1, z0, sign, dtype):
    e = F(x0) + sign * F(y0) - F(z0)
    return gamma(2, dtype) * (abs(F(x1)) + abs(F(y1)) + abs(e))


def bound_mul(x0, x1, y0, y1, z0, dtype):
    e00 = F(x0) * F(y0) - F(z0)
    return gamma(3, dtype) * (abs(e00) + abs(F(x0) * F(y1)) + abs(F(x1) * F(y0)) + abs(F(x1) * F(y1)))


def bound_div(x0, x1, y0, y1, z0, dz0, dtype):
    num = abs(F(x1) - F(z0) * F(y1))
    den = abs(F(y0) + F(y1))
    return gamma(3, dtype) * abs(dz0) + gamma(2, dtype) * num / den


def exact_dz0(op, x0, x1, y0, y1, z0):
    xs, ys = F(x0) + F(x1), F(y0) + F(y1)
    z = {"add": xs + ys, "sub": xs - ys, "mul": xs * ys, "div": xs / ys}[op]
    return z - F(z0)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_general_twofold_bound(op, dtype):
    x0, x1, y0, y1 = _cases(dtype, 21)
    if op == "div":  # keep divisors away from cancellation y0 + y1 ~ 0
        y1 = np.where(np.abs(y1) > 0.25 * np.abs(y0), y1 * np.asarray(0.125, dtype), y1).astype(dtype)
    z0, z1 = getattr(oracle, op)(x0, x1, y0, y1)
    worst = Fraction(0)
    for i in range(N):
        dz0 = exact_dz0(op, x0[i], x1[i], y0[i], y1[i], z0[i])
        if op in ("add", "sub"):
            b = bound_add(x0[i], x1[i], y0[i], y1[i], z0[i], 1 if op == "add" else -1, dtype)
        elif op == "mul":
            b = bound_mul(x0[i], x1[i], y0[i], y1[i], z0[i], dtype)
        else:
            b = bound_div(x0[i], x1[i], y0[i], y1[i], z0[i], dz0, dtype)
        err = abs(F(z1[i]) - dz0)
        assert err <= b, (op, i)
        if b:
            worst = max(worst, err / b)
    assert worst > 0  # the bound is exercised, not vacuous


@pytest.mark.parametrize("dtype", DTYPES)
def test_mul_and_div_with_dotted_divisor(dtype):
    x0, x1, y0, _ = _cases(dtype, 22)
    z0, z1 = oracle.mul(x0, x1, y0, None)
    for i in range(N):
        e00 = F(x0[i]) * F(y0[i]) - F(z0[i])
        dz0 = (F(x0[i]) + F(x1[i])) * F(y0[i]) - F(z0[i])
        assert abs(F(z1[i]) - dz0) <= gamma(2, dtype) * (abs(e00) + abs(F(x1[i]) * F(y0[i])))
    z0, z1 = oracle.div(x0, x1, y0, None)
    for i in range(N):
        dz0 = (F(x0[i]) + F(x1[i])) / F(y0[i]) - F(z0[i])
        assert abs(F(z1[i]) - dz0) <= gamma(2, dtype) * abs(dz0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_div_with_dotted_dividend(dtype):
    """Dotted x over twofold y is DTF1 with x1 = +0 (the overload set lists it
    without a formula): the DTF1 bound with x1 = 0 against the exact dz0.
    A form that ignores y1 is off by about |z0 y1 / y0|, far outside it."""
    x0, _, y0, y1 = _cases(dtype, 23)
    y1 = np.where(np.abs(y1) > 0.25 * np.abs(y0), y1 * np.asarray(0.125, dtype), y1).astype(dtype)
    z0, z1 = oracle.div(x0, None, y0, y1)
    zero = np.zeros(1, dtype)[0]
    worst = Fraction(0)
    for i in range(N):
        assert z0[i] == x0[i] / y0[i]
        dz0 = exact_dz0("div", x0[i], zero, y0[i], y1[i], z0[i])
        b = bound_div(x0[i], zero, y0[i], y1[i], z0[i], dz0, dtype)
        err = abs(F(z1[i]) - dz0)
        assert err <= b, i
        if b:
            worst = max(worst, err / b)
    assert worst > 0


def _mp(v):
    return mpmath.mpf(float(v))


def sqrt_check(x0, x1, z0, z1, dtype, dz_ref=None, slack=0.0):
    """RTF1 bound at one element (see module docstring)."""
    u = float(U[np.dtype(dtype)])
    g2 = float(gamma(2, dtype))
    mpmath.mp.prec = 400
    x = F(x0) + F(x1)
    S = mpmath.sqrt(mpmath.mpf(x.numerator) / x.denominator)
    u0 = rn(x, dtype)
    v0 = mpmath.mpf(float(np.sqrt(u0)))  # correctly rounded root of u0
    delta = abs(S - v0)
    rho = delta / (2 * v0)
    E = delta * (1 + rho) * (g2 + rho / (1 - rho))
    dz0 = S - _mp(z0)
    b = E * (1 + u) + u * (1 + u) * (delta + E + u * abs(v0 - _mp(z0))) + u * abs(dz0)
    ref = dz0 if dz_ref is None else mpmath.mpf(dz_ref)
    return abs(_mp(z1) - ref), b + slack * abs(dz0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_sqrt_bound(dtype):
    x0, x1 = twofold(dtype, N, 23)
    x0 = np.abs(x0)
    x1 = np.where(np.abs(x1) > 0.5 * x0, np.abs(x1), x1).astype(dtype)  # keep x0 + x1 > 0
    z0, z1 = oracle.sqrt(x0, x1)
    for i in range(N):
        err, b = sqrt_check(x0[i], x1[i], z0[i], z1[i], dtype)
        assert err <= b, i


# ---------------------------------------------------------------------------
# composites: running bounds, each step's bound from the list above plus
# the propagated bound of its twofold input
# ---------------------------------------------------------------------------

def axpy_bound(a, x0, x1, y0, y1, z0, dtype):
    """Running bound and exact deviation for one axpy element.
    t = MTF1(a, x): |t1 - dt0| <= B_mul.  z = ATF1(t, y):
    dz0 = dt0 + y1 + e with e = err(t0 + y0), so
    |z1 - dz0| <= B_mul + gamma_2 (|dt0| + B_mul + |y1| + |e|)."""
    a0, a1 = a
    t0 = rn(F(a0) * F(x0), dtype)
    bm = bound_mul(a0, a1, x0, x1, t0, dtype)
    dt0 = (F(a0) + F(a1)) * (F(x0) + F(x1)) - F(t0)
    e = F(t0) + F(y0) - F(z0)
    assert z0 == rn(F(t0) + F(y0), dtype)
    b = bm + gamma(2, dtype) * (abs(dt0) + bm + abs(F(y1)) + abs(e))
    dz0 = (F(a0) + F(a1)) * (F(x0) + F(x1)) + F(y0) + F(y1) - F(z0)
    return b, dz0


def horner_bound(c, x0, x1, z0, dtype):
    """Running bound and exact deviation for one Horner element, through d
    steps of m = MTF1(r, x), r = ATF1.1(m, c_k).  The z0 path is the plain
    Horner recurrence; with B the bound on |r1 - dr0| and r the exact
    partial value,
      mul: |m1 - dm0| <= B |x| + gamma_3 (|e00| + |r0 x1| + (|dr0| + B)(|x0| + |x1|))
      add: |r1' - dr0'| <= B_m + u (|dm0| + B_m + |e|),  e = err(m0 + c_k)."""
    cf = [F(v) for v in c]
    d = len(cf) - 1
    u = U[np.dtype(dtype)]
    g3 = gamma(3, dtype)
    x0, x1 = F(x0), F(x1)
    x = x0 + x1
    r0 = c[d]                # z0 path (binary floating point)
    R = cf[d]                # exact partial value
    B = Fraction(0)
    for k in range(d - 1, -1, -1):
        m0 = rn(F(r0) * x0, dtype)
        e00 = F(r0) * x0 - F(m0)
        dr0 = R - F(r0)
        Bm = B * abs(x) + g3 * (abs(e00) + abs(F(r0) * x1) + (abs(dr0) + B) * (abs(x0) + abs(x1)))
        M = R * x
        dm0 = M - F(m0)
        r0 = rn(F(m0) + cf[k], dtype)
        e = F(m0) + cf[k] - F(r0)
        B = Bm + u * (abs(dm0) + Bm + abs(e))
        R = M + cf[k]
    assert z0 == r0
    return B, R - F(r0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_axpy_bound(dtype):
    from paper_1401_6235_amd import workloads as W
    c = W.axpy_case(N, seed=3, dtype=dtype)
    z0, z1 = oracle.axpy(c["a"], c["x0"], c["x1"], c["y0"], c["y1"])
    for i in range(N):
        b, dz0 = axpy_bound(c["a"], c["x0"][i], c["x1"][i], c["y0"][i], c["y1"][i], z0[i], dtype)
        assert abs(F(z1[i]) - dz0) <= b, i


@pytest.mark.parametrize("dtype", DTYPES)
def test_horner_bound(dtype):
    from paper_1401_6235_amd import workloads as W
    n = 300
    c = W.horner_case(n, seed=4, dtype=dtype)
    z0, z1 = oracle.horner(c["c"], c["x0"], c["x1"])
    for i in range(n):
        b, dz0 = horner_bound(c["c"], c["x0"][i], c["x1"][i], z0[i], dtype)
        assert abs(F(z1[i]) - dz0) <= b, i


# ---------------------------------------------------------------------------
# binary32 twofolds judged by the binary64 oracle
# ---------------------------------------------------------------------------

REF_SLACK = Fraction(1, 2 ** 50)


def magnitude(op, x0, x1, y0, y1, z0, dz0):
    """The quantity M that each binary bound multiplies by gamma_k (with
    |dz0| added for division)."""
    if op in ("add", "sub"):
        sign = 1 if op == "add" else -1
        return abs(F(x1)) + abs(F(y1)) + abs(F(x0) + sign * F(y0) - F(z0))
    if op == "mul":
        e00 = F(x0) * F(y0) - F(z0)
        return abs(e00) + abs(F(x0) * F(y1)) + abs(F(x1) * F(y0)) + abs(F(x1) * F(y1))
    return abs(dz0) + abs(F(x1) - F(z0) * F(y1)) / abs(F(y0) + F(y1))


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_fp32_against_fp64_reference(op):
    """The binary64 reference runs the same algorithm with u = 2^-53 on the
    widened operands; its rounding errors never exceed the binary32 ones
    (the nearest double is at least as near as the nearest float), so it is
    within 2^-50 (M + |dz0|) of the exact deviation, and the binary32 z1 is
    judged by its binary32 bound plus that slack."""
    from paper_1401_6235_amd import workloads as W
    c = W.elementwise(op, N, seed=0, dtype=np.float32)
    x0, x1, y0, y1 = c["x0"], c["x1"], c["y0"], c["y1"]
    z0, z1 = getattr(oracle, op)(x0, x1, y0, y1)
    dz = oracle.ref64(op, x0, x1, y0, y1, z0)
    dt = np.float32
    for i in range(N):
        ref = F(dz[i])
        exact = exact_dz0(op, x0[i], x1[i], y0[i], y1[i], z0[i])
        M = magnitude(op, x0[i], x1[i], y0[i], y1[i], z0[i], exact)
        assert abs(ref - exact) <= REF_SLACK * (M + abs(exact)), (op, i)
        if op in ("add", "sub"):
            b = bound_add(x0[i], x1[i], y0[i], y1[i], z0[i], 1 if op == "add" else -1, dt)
        elif op == "mul":
            b = bound_mul(x0[i], x1[i], y0[i], y1[i], z0[i], dt)
        else:
            b = bound_div(x0[i], x1[i], y0[i], y1[i], z0[i], ref, dt)
        assert abs(F(z1[i]) - ref) <= b + REF_SLACK * (M + abs(ref)), (op, i)


def test_fp32_sqrt_against_fp64_reference():
    from paper_1401_6235_amd import workloads as W
    c = W.elementwise("sqrt", N, seed=0, dtype=np.float32)
    z0, z1 = oracle.sqrt(c["x0"], c["x1"])
    dz = oracle.ref64("sqrt", c["x0"], c["x1"], z0)
    for i in range(N):
        err, b = sqrt_check(c["x0"][i], c["x1"][i], z0[i], z1[i], np.float32, dz_ref=dz[i],
                            slack=float(REF_SLACK))
        assert err <= b, i


def test_fp32_composites_against_fp64_reference():
    """axpy / Horner in binary32 against the binary64 reference.  The
    binary64 run takes the same steps with rounding errors no larger than
    the binary32 ones, so it is within 2^-28 B32 + 2^-52 |dz0| of the exact
    deviation (B32 the binary32 running bound, scaled by u64/u32 = 2^-29
    with a factor 2 to spare)."""
    from paper_1401_6235_amd import workloads as W
    n = 300
    f32 = np.float32
    c = W.axpy_case(n, seed=3, dtype=f32)
    z0, z1 = oracle.axpy(c["a"], c["x0"], c["x1"], c["y0"], c["y1"])
    dz = oracle.ref64("axpy", c["a"], c["x0"], c["x1"], c["y0"], c["y1"], z0)
    for i in range(n):
        b, exact = axpy_bound(c["a"], c["x0"][i], c["x1"][i], c["y0"][i], c["y1"][i], z0[i], f32)
        slack = b / 2 ** 28 + abs(exact) / 2 ** 52
        assert abs(F(dz[i]) - exact) <= slack, i
        assert abs(F(z1[i]) - F(dz[i])) <= b + 2 * slack, i
    h = W.horner_case(n, seed=4, dtype=f32)
    z0, z1 = oracle.horner(h["c"], h["x0"], h["x1"])
    dz = oracle.ref64("horner", h["c"], h["x0"], h["x1"], z0)
    for i in range(n):
        b, exact = horner_bound(h["c"], h["x0"][i], h["x1"][i], z0[i], f32)
        slack = b / 2 ** 28 + abs(exact) / 2 ** 52
        assert abs(F(dz[i]) - exact) <= slack, i
        assert abs(F(z1[i]) - F(dz[i])) <= b + 2 * slack, i
