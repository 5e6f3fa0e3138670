"""GPU parity: twofold sum and dot, bit for bit against the oracle's tree.

Covers every leaf kind (dotted and twofold sums; dotted, twofold and mixed
dots; plain sum and dot), sizes from 0 to the full n = 2^26 instances of
the ill-conditioned dot generator (condition numbers 1e4 .. 1e32 in
binary64, 1e4 .. 1e16 in binary32), ragged tails, misaligned views, and
every reduction block geometry (the tree must not depend on it), and sizes
around the tuned shapes' block boundaries.
"""
import numpy as np
import pytest

import oracle
import paper_1401_6235_amd as tf
from gpu_util import assert_bits, step, to_gpu, to_np, torch_cuda
from paper_1401_6235_amd import workloads as W

pytestmark = pytest.mark.gpu

DTYPES = [np.float64, np.float32]
SIZES = [0, 1, 2, 3, 4, 5, 255, 256, 257, 1000, 4096, 4099, 65536, 65537, 300001, 1 << 20, 5000011]


def gpu_all(x0, x1, y0, y1):
    g = [to_gpu(v) for v in (x0, x1, y0, y1)]
    out = {
        "sum_t": to_np(tf.tf_sum(g[0], g[1])),
        "sum_d": to_np(tf.tf_sum(g[0])),
        "dot_dd": to_np(tf.tf_dot(g[0], None, g[2], None)),
        "dot_tt": to_np(tf.tf_dot(g[0], g[1], g[2], g[3])),
        "dot_td": to_np(tf.tf_dot(g[0], g[1], g[2], None)),
        "dot_dt": to_np(tf.tf_dot(g[0], None, g[2], g[3])),
        "psum": to_np(tf.tf_plain_sum(g[0])),
        "pdot": to_np(tf.tf_plain_dot(g[0], g[2])),
    }
    return out


def oracle_all(x0, x1, y0, y1):
    return {
        "sum_t": np.array(oracle.sum(x0, x1)),
        "sum_d": np.array(oracle.sum(x0)),
        "dot_dd": np.array(oracle.dot(x0, None, y0, None)),
        "dot_tt": np.array(oracle.dot(x0, x1, y0, y1)),
        "dot_td": np.array(oracle.dot(x0, x1, y0, None)),
        "dot_dt": np.array(oracle.dot(x0, None, y0, y1)),
        "psum": np.array([oracle.plain_sum(x0)]),
        "pdot": np.array([oracle.plain_dot(x0, y0)]),
    }


def random_case(n, dtype, seed):
    g = np.random.default_rng(seed)
    x0 = (g.standard_normal(n) * np.exp2(g.integers(-30, 30, n))).astype(dtype)
    y0 = (g.standard_normal(n) * np.exp2(g.integers(-30, 30, n))).astype(dtype)
    x1 = (x0.astype(np.float64) * g.uniform(-1, 1, n) * 2.0 ** -20).astype(dtype)
    y1 = (y0.astype(np.float64) * g.uniform(-1, 1, n) * 2.0 ** -20).astype(dtype)
    return x0, x1, y0, y1


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SIZES)
def test_all_leaf_kinds(n, dtype):
    step("reduce n=%d %s" % (n, np.dtype(dtype)))
    case = random_case(n, dtype, n + 1)
    got, want = gpu_all(*case), oracle_all(*case)
    for k in want:
        assert_bits(got[k], want[k], "%s n=%d" % (k, n))


def _boundary_sizes():
    """Sizes around the tuned first-pass shapes' block boundaries: tile
    counts at small multiples of 32, 64 and 128 tiles and one tile or one
    leaf either side (every third of them, to bound the oracle's time)."""
    sizes = set()
    for pb in (32, 64, 128):
        for m in (1, 2, 3, 7, 63, 64, 65):
            for d in (-257, -1, 0, 1, 255, 256, 257):
                sizes.add(pb * m * 256 + d)
    return sorted(sizes)[::3]


@pytest.mark.parametrize("dtype", DTYPES)
def test_tuned_shape_block_boundaries(dtype):
    for n in _boundary_sizes():
        step("shape boundary n=%d %s" % (n, np.dtype(dtype)))
        case = random_case(n, dtype, n % 9973)
        got, want = gpu_all(*case), oracle_all(*case)
        for k in want:
            assert_bits(got[k], want[k], "%s n=%d" % (k, n))


@pytest.mark.parametrize("dtype", DTYPES)
def test_every_block_geometry_gives_the_same_bits(dtype):
    n = 3 * (1 << 18) + 77
    case = random_case(n, dtype, 99)
    want = oracle_all(*case)
    # tiles per block at the tuned waves, then every wave count (4, 8, 16;
    # the one-pass kernel where each wave takes exactly one tile group)
    geometries = [(tpb, 0) for tpb in (1, 2, 4, 8, 16, 32, 64, 128, 256)]
    geometries += [(tpb, wv) for wv in (4, 8, 16) for tpb in (8, 16, 32, 64, 256)]
    for tpb, wv in geometries:
        step("geometry tiles/block=%d waves=%d %s" % (tpb, wv, np.dtype(dtype)))
        old = tf.tf_config(tf.TF_CFG_RED_TILES_PER_BLOCK, tpb)
        old_w = tf.tf_config(tf.TF_CFG_RED_WAVES, wv)
        try:
            got = gpu_all(*case)
        finally:
            tf.tf_config(tf.TF_CFG_RED_TILES_PER_BLOCK, old)
            tf.tf_config(tf.TF_CFG_RED_WAVES, old_w)
        for k in want:
            assert_bits(got[k], want[k], "%s tpb=%d waves=%d" % (k, tpb, wv))


@pytest.mark.parametrize("dtype", DTYPES)
def test_misaligned_and_special(dtype):
    torch = torch_cuda()
    n = 70001
    x0, x1, y0, y1 = random_case(n + 1, dtype, 5)
    x0[17] = np.inf
    y0[5000] = -0.0
    x1[9] = np.nan
    g = [to_gpu(v)[1:] for v in (x0, x1, y0, y1)]
    step("misaligned reduce %s" % np.dtype(dtype))
    got = to_np(tf.tf_dot(g[0], g[1], g[2], g[3]))
    assert_bits(got, np.array(oracle.dot(x0[1:], x1[1:], y0[1:], y1[1:])), "dot")
    got = to_np(tf.tf_sum(g[0], None))
    assert_bits(got, np.array(oracle.sum(x0[1:])), "sum")
    torch.cuda.synchronize()


@pytest.mark.parametrize("cond", [1e4, 1e8, 1e16, 1e32])
def test_full_size_ill_conditioned_f64(cond):
    """n = 2^26 binary64: dot of the generator's (x, y) and sum of the exact
    product split, checked whole against the oracle."""
    n = 1 << 26
    step("illdot f64 n=2^26 cond=%g (generate)" % cond)
    d = W.illdot_case(n, cond, seed=0, dtype=np.float64)
    hi, lo = W.product_split(d["x"], d["y"])
    step("illdot f64 n=2^26 cond=%g (run)" % cond)
    gx, gy, ghi, glo = (to_gpu(v) for v in (d["x"], d["y"], hi, lo))
    assert_bits(to_np(tf.tf_dot(gx, None, gy, None)), np.array(oracle.dot(d["x"], None, d["y"], None)), "dot")
    assert_bits(to_np(tf.tf_sum(ghi, glo)), np.array(oracle.sum(hi, lo)), "sum")
    assert_bits(to_np(tf.tf_plain_dot(gx, gy)), np.array([oracle.plain_dot(d["x"], d["y"])]), "plain dot")


def tree_depth(n):
    """Levels of the reduction tree: 8 inside a 256-leaf tile, then one per
    doubling of the padded tile count."""
    tiles = max(1, -(-n // 256))
    return 8 + (tiles - 1).bit_length()


def tree_bound(n, u, A, lam=None):
    """|z0 + z1 - exact| for the twofold tree over leaves (L0, L1) with
    |L1| <= lam |L0 + L1|: a node's rounding error e is exact and z1 gathers
    the leaves' low parts and the node errors with two roundings per node.
    With lam <= u (Two-Product leaves, an exact product split in the same
    format) that is (d^2 + 4d) u^2 sum|leaf| to first order; a larger lam
    adds 2 d u lam sum|leaf| (the low parts rounded once per level).  A
    factor 2 covers the higher-order terms."""
    d = tree_depth(n)
    b = (d * d + 4 * d) * u * u * A
    if lam is not None and lam > u:
        b += 2 * d * u * lam * A
    return 2 * b


@pytest.mark.parametrize("cond", [1e4, 1e8, 1e16])
def test_full_size_ill_conditioned_f32(cond):
    """n = 2^26 binary32, bit for bit against the oracle; then z0 + z1
    against the exact dot (the generator's fixed-point accumulator, rounded
    once to binary64) within the tree bound at u = 2^-24, and z1 against the
    binary64 reference deviation of z0 within the same bound plus the
    reference's own error: the tree bound at u = 2^-53 (the widened dot's
    products are exact; the widened sum's leaves keep low parts up to
    2^-24 of their value), doubled, and two binary64 roundings of the
    deviation."""
    from fractions import Fraction as Fr
    n = 1 << 26
    u32, u64 = 2.0 ** -24, 2.0 ** -53
    step("illdot f32 n=2^26 cond=%g" % cond)
    d = W.illdot_case(n, cond, seed=0, dtype=np.float32)
    hi, lo = W.product_split(d["x"], d["y"])
    gx, gy, ghi, glo = (to_gpu(v) for v in (d["x"], d["y"], hi, lo))
    dot = to_np(tf.tf_dot(gx, None, gy, None))
    assert_bits(dot, np.array(oracle.dot(d["x"], None, d["y"], None)), "dot")
    s = to_np(tf.tf_sum(ghi, glo))
    assert_bits(s, np.array(oracle.sum(hi, lo)), "sum")
    del gx, gy, ghi, glo
    x64, y64 = d["x"].astype(np.float64), d["y"].astype(np.float64)
    exact = W.exact_dot_f64(x64, y64)  # x^T y rounded once
    A = float(np.abs(x64 * y64).sum()) * (1 + 2.0 ** -20)  # products exact; sum to 2^-27
    b32 = tree_bound(n, u32, A)
    for name, z, dz, lam in (("dot", dot, oracle.ref64("dot", d["x"], None, d["y"], None, dot[0]), 0.0),
                             ("sum", s, oracle.ref64("sum", hi, lo, s[0]), u32)):
        got = Fr(float(z[0])) + Fr(float(z[1]))
        assert abs(got - Fr(exact)) <= Fr(b32) + Fr(u64 * abs(exact)), (name, cond)
        ref_err = 2 * tree_bound(n, u64, A, lam) + 4 * u64 * abs(float(dz[0]))
        assert abs(Fr(float(z[1])) - Fr(float(dz[0]))) <= Fr(b32) + Fr(ref_err), (name, cond)
        # the reference itself is within its error of the exact deviation
        assert abs(Fr(float(dz[0])) - (Fr(exact) - Fr(float(z[0])))) <= Fr(ref_err) + Fr(u64 * abs(exact))


def test_repeat_is_bitwise_stable():
    case = random_case(1 << 22, np.float64, 3)
    step("repeat determinism")
    a = gpu_all(*case)
    b = gpu_all(*case)
    for k in a:
        assert_bits(a[k], b[k], k)


@pytest.mark.parametrize("dtype", DTYPES)
def test_side_stream_with_binding_workspace(dtype):
    """tf_sum / tf_dot on a side stream (stream=) with the workspace and
    output made by the binding.  The side stream is held back by copies
    queued first; right after the calls return, the current stream
    allocates buffers of the workspace's size and fills them.  A workspace
    handed to those allocations would be overwritten before the reduction
    reads its partials."""
    torch = torch_cuda()
    n = 3000017
    case = random_case(n, dtype, 123)
    g = [to_gpu(v) for v in case]
    big = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
    big_out = torch.empty_like(big)
    cur = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    side.wait_stream(cur)
    step("side-stream reductions %s" % np.dtype(dtype))
    for _ in range(8):
        tf.tf_vmem(big, big, big_out, stream=side)
    s = tf.tf_sum(g[0], g[1], stream=side)
    d = tf.tf_dot(g[0], None, g[2], None, stream=side)
    ws = tf.tf_reduce_workspace_bytes(tf.TF_F64 if dtype == np.float64 else tf.TF_F32, n)
    junk = [torch.full((ws,), 255, dtype=torch.uint8, device="cuda") for _ in range(8)]
    torch.cuda.synchronize()
    assert_bits(to_np(s), np.array(oracle.sum(case[0], case[1])), "sum on a side stream")
    assert_bits(to_np(d), np.array(oracle.dot(case[0], None, case[2], None)), "dot on a side stream")
    del junk, big, big_out


def test_workspace_too_small_is_an_error():
    torch = torch_cuda()
    x = torch.ones(100000, dtype=torch.float64, device="cuda")
    with pytest.raises(tf.TwofoldError):
        tf.tf_sum(x, None, work=torch.empty(8, dtype=torch.uint8, device="cuda"))
