"""The oracle's twofold sum and dot (no GPU).

The reduction is a fixed pairwise tree over element indices: 256-leaf
tiles, zero-padded, then the tile results paired the same way up to a power
of two.  Every node is ATF1; a twofold accumulator over plain numbers is
the use the paper singles out as sound (the 2x section).

Pins:
  * z0 is the standard pairwise sum (an independent numpy evaluation of the
    same complete tree), bitwise;
  * z0 + z1 is within (d^2 + 4d) u^2 sum|leaf| of the exact sum, d the tree
    depth (each node's error term is exact; z1 sums them with two roundings
    per node), checked against exact rational dots of ill-conditioned
    instances with condition numbers 1e4 ... 1e32 (margin 2);
  * n = 0 gives (+0, +0); one product gives the exact Two-Product; two
    dotted values give the exact Two-Sum;
  * the dot of plain vectors equals the sum of the exact product split of
    its terms, bitwise; appending zeros that stay inside the padding does not
    change a bit.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact import F, U, bits_equal
from paper_1401_6235_amd import workloads as W

DTYPES = [np.float64, np.float32]
SIZES = [0, 1, 2, 3, 255, 256, 257, 511, 1000, 4096, 4099, 70001]


def plain_tree(leaves):
    """The standard (plain) pairwise sum over the padded complete tree,
    evaluated level by level with numpy."""
    leaves = np.asarray(leaves)
    n = leaves.size
    if n == 0:
        return leaves.dtype.type(0)
    tiles = -(-n // 256)
    padded = 1 << (tiles - 1).bit_length()
    buf = np.zeros(padded * 256, leaves.dtype)
    buf[:n] = leaves
    while buf.size > 1:
        buf = buf[0::2] + buf[1::2]
    return buf[0]


def depth(n):
    tiles = max(1, -(-n // 256))
    return 8 + (tiles - 1).bit_length()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SIZES)
def test_z0_is_the_plain_pairwise_sum(n, dtype):
    g = np.random.default_rng(n + 7)
    x0 = (g.standard_normal(n) * np.exp2(g.integers(-10, 10, n))).astype(dtype)
    x1 = (x0 * g.uniform(-1, 1, n) * 2.0 ** -30).astype(dtype)
    y0 = g.standard_normal(n).astype(dtype)
    y1 = (y0 * g.uniform(-1, 1, n) * 2.0 ** -30).astype(dtype)
    z = oracle.sum(x0, x1)
    assert bits_equal(z[0], plain_tree(x0))
    assert bits_equal(z[0], oracle.plain_sum(x0))
    z = oracle.sum(x0)
    assert bits_equal(z[0], plain_tree(x0))
    for a1, b1 in ((None, None), (x1, y1), (x1, None), (None, y1)):
        z = oracle.dot(x0, a1, y0, b1)
        assert bits_equal(z[0], plain_tree(x0 * y0))
    assert bits_equal(oracle.plain_dot(x0, y0), plain_tree(x0 * y0))


@pytest.mark.parametrize("dtype", DTYPES)
def test_degenerate_sizes(dtype):
    e = np.zeros(0, dtype)
    for z in (oracle.sum(e), oracle.sum(e, e), oracle.dot(e, None, e, None), oracle.dot(e, e, e, e)):
        assert z[0] == 0 and z[1] == 0
        assert not np.signbit(z[0]) and not np.signbit(z[1])
    g = np.random.default_rng(3)
    for _ in range(200):
        a, b = g.standard_normal(2).astype(dtype) * dtype(1e3)
        z = oracle.dot(np.array([a]), None, np.array([b]), None)
        assert F(z[0]) + F(z[1]) == F(a) * F(b)            # Two-Product leaf
        z = oracle.sum(np.array([a, b]))
        assert F(z[0]) + F(z[1]) == F(a) + F(b)            # Two-Sum at level 1


@pytest.mark.parametrize("dtype", DTYPES)
def test_zero_padding_is_invisible(dtype):
    g = np.random.default_rng(4)
    x = g.standard_normal(1000).astype(dtype)
    y = g.standard_normal(1000).astype(dtype)
    for k in (1, 24):  # 1000 + k stays inside the same 1024-leaf tree
        xz = np.concatenate([x, np.zeros(k, dtype)])
        yz = np.concatenate([y, np.zeros(k, dtype)])
        assert bits_equal(np.array(oracle.dot(x, None, y, None)), np.array(oracle.dot(xz, None, yz, None))).all()
        assert bits_equal(np.array(oracle.sum(x)), np.array(oracle.sum(xz))).all()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("cond", [1e4, 1e8, 1e16, 1e32])
def test_dot_against_exact_rational(cond, dtype):
    n = 1 << 12
    d = W.illdot_case(n, cond, seed=0, dtype=dtype)
    x, y = d["x"], d["y"]
    z0, z1 = oracle.dot(x, None, y, None)
    exact = sum(F(a) * F(b) for a, b in zip(x, y))
    A = sum(abs(F(a) * F(b)) for a, b in zip(x, y))
    dd = depth(n)
    u = U[np.dtype(dtype)]
    bound = 2 * (dd * dd + 4 * dd) * u * u * A
    assert abs(F(z0) + F(z1) - exact) <= bound
    # the same instance as twofold leaves (exact product split) sums to the
    # same bits
    hi, lo = W.product_split(x, y)
    s = oracle.sum(hi, lo)
    assert bits_equal(s[0], z0) and bits_equal(s[1], z1)
    # and its dotted sum of the rounded products is pinned the same way
    s0, s1 = oracle.sum(hi)
    exact_hi = sum(F(v) for v in hi)
    Ahi = sum(abs(F(v)) for v in hi)
    assert abs(F(s0) + F(s1) - exact_hi) <= bound * Ahi / A + 2 * (dd * dd + 4 * dd) * u * u * Ahi


@pytest.mark.parametrize("dtype", DTYPES)
def test_twofold_dot_bound(dtype):
    """Twofold inputs: MTF1 leaves carry their own error (gamma_3 of their
    terms), then the tree bound applies."""
    n = 3000
    g = np.random.default_rng(9)
    x0 = g.standard_normal(n).astype(dtype)
    y0 = g.standard_normal(n).astype(dtype)
    x1 = (x0 * g.uniform(-1, 1, n) * 2.0 ** -12).astype(dtype)
    y1 = (y0 * g.uniform(-1, 1, n) * 2.0 ** -12).astype(dtype)
    z0, z1 = oracle.dot(x0, x1, y0, y1)
    u = U[np.dtype(dtype)]
    exact = Fraction(0)
    A = Fraction(0)
    leaf = Fraction(0)
    for i in range(n):
        xs, ys = F(x0[i]) + F(x1[i]), F(y0[i]) + F(y1[i])
        exact += xs * ys
        A += abs(xs * ys)
        p = F(x0[i]) * F(y0[i])
        leaf += 3 * u * (u * abs(p) + abs(F(x0[i]) * F(y1[i])) + abs(F(x1[i]) * F(y0[i]))
                         + abs(F(x1[i]) * F(y1[i])))
    dd = depth(n)
    bound = leaf * (1 + 4 * u * dd) + 2 * (dd * dd + 4 * dd) * u * u * A * 2
    assert abs(F(z0) + F(z1) - exact) <= bound


@pytest.mark.parametrize("dtype", DTYPES)
def test_exact_partial_sums_give_zero_error(dtype):
    """Small integers: every node sums exactly, so z1 is zero and z0 exact."""
    g = np.random.default_rng(5)
    x = g.integers(-1000, 1000, 5000).astype(dtype)
    z0, z1 = oracle.sum(x)
    assert z0 == x.astype(np.float64).sum() and z1 == 0
    y = g.integers(-3, 4, 5000).astype(dtype)
    z0, z1 = oracle.dot(x, None, y, None)
    assert z0 == float(np.dot(x.astype(np.int64), y.astype(np.int64))) and z1 == 0
