"""Batched applications and the twofold fma in the oracle (no GPU).

Pins, each independent of the code under test:

* Back-substitution: the paper's 3x3 Jordan-block logs (Applications,
  Linear Ax=f) reproduced through the batched solver, many systems at once
  in the interleaved layout; upper-triangular integer systems with
  power-of-two diagonals have exact solutions, so x0 is exact and x1 is 0;
  a dotted matrix gives the values of a twofold one with zero low parts.
* Quadratic: the paper's logs (Applications, Square root), with the float
  row's error signs negated as the sign reading of Algorithm 2.2 implies,
  and its NaN flow when the discriminant is negative; integer roots are
  found exactly with zero error parts.
* fma: z0 is the hardware fma; the rounded error of that fma is
  RN(x0 y0 + w0 - z0) exactly (Boldo and Muller's ErrFma gives the error
  as an exact sum r2 + r3 with r2 the rounded sum), checked in rational
  arithmetic; with w = 0 it reduces to MTF1 and with x = 1 to the Two-Sum
  residual.  The remaining terms round at most four times:
  |z1 - dz0| <= gamma_4 (|err| + |x1 y1| + |x0 y1| + |x1 y0| + |w1|).
"""
import numpy as np
import pytest

import oracle
from exact import F, bits_equal, gamma, rn
from test_oracle_eft import twofold
from test_oracle_paper import LOGS, TYPES, close6, parse, twofold_of_double

DTYPES = [np.float64, np.float32]


# ---- back-substitution --------------------------------------------------------

def jordan_batch(runs, dt):
    """The paper's 3x3 Jordan blocks, one system per run, interleaved."""
    m, ns = 3, len(runs)
    U0 = np.zeros(m * m * ns, dt)
    U1 = np.zeros(m * m * ns, dt)
    f0 = np.zeros(m * ns, dt)
    for k, run in enumerate(runs):
        lam = twofold_of_double(run["lambda"], dt)
        for i in range(m):
            U0[(i * m + i) * ns + k], U1[(i * m + i) * ns + k] = lam
            if i + 1 < m:
                U0[(i * m + i + 1) * ns + k] = 1
            f0[i * ns + k] = run["f"][i]
    return U0, U1, f0


@pytest.mark.parametrize("type_name", ["float", "double"])
def test_jordan_block_logs_through_the_batched_solver(type_name):
    dt = TYPES[type_name]
    runs = [r for r in LOGS["gauss"]["runs"] if r["type"] == type_name]
    U0, U1, f0 = jordan_batch(runs, dt)
    x0, x1 = oracle.trsv_upper(3, U0, U1, f0, np.zeros_like(f0))
    ns = len(runs)
    for k, run in enumerate(runs):
        for i in range(3):
            p0, p1 = parse(run["x"][i])
            assert close6(x0[i * ns + k], p0), (run["lambda"], i)
            assert close6(x1[i * ns + k], p1), (run["lambda"], i)


def integer_systems(dt, m, nsys, seed):
    """Upper-triangular U with power-of-two diagonal and small integers above
    it, and f = U x for an integer x: every step is exact."""
    g = np.random.default_rng(seed)
    U = np.zeros((m, m, nsys))
    for i in range(m):
        U[i, i] = np.exp2(g.integers(-2, 3, nsys)) * np.where(g.integers(0, 2, nsys) == 1, -1, 1)
        for j in range(i + 1, m):
            U[i, j] = g.integers(-3, 4, nsys)
    x = g.integers(-9, 10, (m, nsys)).astype(np.float64)
    f = np.einsum("ijk,jk->ik", U, x)
    return U.reshape(-1).astype(dt), f.reshape(-1).astype(dt), x.reshape(-1)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m", [1, 4, 9])
def test_exact_systems_are_solved_exactly(m, dtype):
    U0, f0, x = integer_systems(dtype, m, 300, 70 + m)
    for U1 in (np.zeros_like(U0), None):
        x0, x1 = oracle.trsv_upper(m, U0, U1, f0, None)
        assert (x0 == x).all()
        assert (x1 == 0).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_one_by_one_system_is_the_division(dtype):
    a0, a1 = twofold(dtype, 500, 73)
    f0, f1 = twofold(dtype, 500, 74)
    x = oracle.trsv_upper(1, a0, a1, f0, f1)
    want = oracle.div(f0, f1, a0, a1)
    assert bits_equal(x[0], want[0]).all() and bits_equal(x[1], want[1]).all()
    x = oracle.trsv_upper(1, a0, None, f0, f1)
    want = oracle.div(f0, f1, a0, None)
    assert bits_equal(x[0], want[0]).all() and bits_equal(x[1], want[1]).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_dotted_matrix_matches_zero_low_parts(dtype):
    g = np.random.default_rng(75)
    m, ns = 6, 400
    U0 = g.uniform(-1, 1, m * m * ns).astype(dtype)
    for i in range(m):
        U0[(i * m + i) * ns:(i * m + i + 1) * ns] += dtype(4)
    f0, f1 = twofold(dtype, m * ns, 76)
    a = oracle.trsv_upper(m, U0, None, f0, f1)
    b = oracle.trsv_upper(m, U0, np.zeros_like(U0), f0, f1)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


# ---- quadratic -------------------------------------------------------------------

@pytest.mark.parametrize("run", LOGS["quadratic"]["runs"], ids=lambda r: "%s-%s" % (r["type"], r["c"]))
def test_quadratic_logs_through_the_batched_solver(run):
    dt = TYPES[run["type"]]
    c64 = {"1e-08": 1e-08, "1+1e-08": 1 + 1e-08}[run["c"]]
    c = twofold_of_double(c64, dt)
    one = lambda v: np.asarray([v], dt)  # noqa: E731
    r0, r1, s0, s1 = oracle.quadratic(one(1), one(0), one(2), one(0), one(c[0]), one(c[1]))
    sign = -1.0 if run["negated_error_sign"] else 1.0
    for name, got in (("x0", (r0[0], r1[0])), ("x1", (s0[0], s1[0]))):
        p0, p1 = parse(run[name])
        assert close6(got[0], p0), (name, got)
        assert close6(got[1], sign * p1), (name, got)


@pytest.mark.parametrize("dtype", DTYPES)
def test_integer_roots_are_exact(dtype):
    g = np.random.default_rng(77)
    p = g.integers(-50, 51, 500).astype(np.float64)
    q = g.integers(-50, 51, 500).astype(np.float64)
    z = np.zeros(500, dtype)
    r0, r1, s0, s1 = oracle.quadratic(np.ones(500, dtype), z, (-(p + q)).astype(dtype), z, (p * q).astype(dtype), z)
    assert (r0 == np.minimum(p, q)).all() and (s0 == np.maximum(p, q)).all()
    # a double root has discriminant 0, and RTF1 at 0 gives 0 / 0 in its
    # low part (the literal formula): the error parts are NaN there
    simple = p != q
    assert simple.sum() > 400 and (~simple).sum() > 0
    assert (r1[simple] == 0).all() and (s1[simple] == 0).all()
    assert np.isnan(r1[~simple]).all() and np.isnan(s1[~simple]).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_negative_discriminant_flows_as_nan(dtype):
    g = np.random.default_rng(78)
    b = g.uniform(-2, 2, 300).astype(dtype)
    c = (b.astype(np.float64) ** 2 / 4 + g.uniform(0.1, 3, 300)).astype(dtype)
    z = np.zeros(300, dtype)
    r0, r1, s0, s1 = oracle.quadratic(np.ones(300, dtype), z, b, z, c, z)
    assert np.isnan(r1).all() and np.isnan(s1).all()
    assert np.isnan(r0).all() and np.isnan(s0).all()


# ---- fma --------------------------------------------------------------------------

def fma_operands(dtype, n, seed, spread):
    x0, x1 = twofold(dtype, n, seed)
    y0, y1 = twofold(dtype, n, seed + 1)
    w0, w1 = twofold(dtype, n, seed + 2)
    g = np.random.default_rng(seed + 3)
    # put the addend near -x0 y0 for a part of the cases: cancellation
    near = g.integers(0, 3, n) == 0
    w0 = np.where(near, (-(x0.astype(np.float64) * y0.astype(np.float64))
                         * (1 + g.uniform(-spread, spread, n))), w0).astype(dtype)
    return x0, x1, y0, y1, w0, w1


@pytest.mark.parametrize("dtype", DTYPES)
def test_fma_error_is_rounded_exactly(dtype):
    x0, _, y0, _, w0, _ = fma_operands(dtype, 3000, 80, 1e-3)
    z0, z1 = oracle.fma(x0, None, y0, None, w0, None)
    for i in range(x0.size):
        assert z0[i] == rn(F(x0[i]) * F(y0[i]) + F(w0[i]), dtype), i
        err = F(x0[i]) * F(y0[i]) + F(w0[i]) - F(z0[i])
        assert z1[i] == rn(err, dtype), i


@pytest.mark.parametrize("dtype", DTYPES)
def test_fma_without_addend_is_mtf1(dtype):
    x0, x1 = twofold(dtype, 1000, 84)
    y0, y1 = twofold(dtype, 1000, 85)
    z = np.zeros_like(x0)
    a = oracle.fma(x0, x1, y0, y1, z, None)
    b = oracle.mul(x0, x1, y0, y1)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
    a = oracle.fma(x0, x1, y0, None, z, None)
    b = oracle.mul(x0, x1, y0, None)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


@pytest.mark.parametrize("dtype", DTYPES)
def test_fma_with_unit_factor_is_two_sum(dtype):
    y0, _ = twofold(dtype, 1000, 86)
    w0, _ = twofold(dtype, 1000, 87)
    a = oracle.fma(np.ones_like(y0), None, y0, None, w0, None)
    b = oracle.two_sum(y0, w0)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("forms", ["ttt", "tdt", "dtd", "ddt"])
def test_fma_bound(forms, dtype):
    x0, x1, y0, y1, w0, w1 = fma_operands(dtype, 2000, 90, 1e-6)
    x1 = x1 if forms[0] == "t" else None
    y1 = y1 if forms[1] == "t" else None
    w1 = w1 if forms[2] == "t" else None
    z0, z1 = oracle.fma(x0, x1, y0, y1, w0, w1)
    lo = lambda v, i: F(v[i]) if v is not None else 0  # noqa: E731
    for i in range(x0.size):
        X0, X1, Y0, Y1, W1 = F(x0[i]), lo(x1, i), F(y0[i]), lo(y1, i), lo(w1, i)
        err = X0 * Y0 + F(w0[i]) - F(z0[i])
        dz0 = err + X0 * Y1 + X1 * Y0 + X1 * Y1 + W1
        b = gamma(4, dtype) * (abs(err) + abs(X1 * Y1) + abs(X0 * Y1) + abs(X1 * Y0) + abs(W1))
        assert abs(F(z1[i]) - dz0) <= b, i
