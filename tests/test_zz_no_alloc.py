"""GPU: tf_dot_noalloc (partials in the library's static device array)
against tf_dot (caller workspace), bit for bit, through the C ABI.

Two calls in a row on one stream, the second smaller, for every leaf kind
and both types; a size whose partials take two levels; n = 0; a tiling
whose partials would not fit (the call adapts it); and the rejection of a
size whose partials cannot fit.  Run after the other GPU
tests and alone in a fresh process, it must pass either way.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1401_6235_amd as tf
from gpu_util import assert_bits, step, to_gpu, to_np, torch_cuda

pytestmark = pytest.mark.gpu

DTYPES = [np.float64, np.float32]
KINDS = {"dd": (False, False), "tt": (True, True), "td": (True, False), "dt": (False, True)}


def random_case(n, dtype, seed):
    g = np.random.default_rng(seed)
    x0 = (g.standard_normal(n) * np.exp2(g.integers(-30, 30, n))).astype(dtype)
    y0 = (g.standard_normal(n) * np.exp2(g.integers(-30, 30, n))).astype(dtype)
    x1 = (x0.astype(np.float64) * g.uniform(-1, 1, n) * 2.0 ** -20).astype(dtype)
    y1 = (y0.astype(np.float64) * g.uniform(-1, 1, n) * 2.0 ** -20).astype(dtype)
    return x0, x1, y0, y1


def pick(case, kind):
    xt, yt = KINDS[kind]
    x0, x1, y0, y1 = case
    return x0, (x1 if xt else None), y0, (y1 if yt else None)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", list(KINDS))
def test_two_calls_in_a_row_match_tf_dot(kind, dtype):
    torch = torch_cuda()
    n1, n2 = 3 * (1 << 18) + 77, 4099
    a = pick(random_case(n1, dtype, 7), kind)
    b = pick(random_case(n2, dtype, 8), kind)
    ga = [to_gpu(v) for v in a]
    gb = [to_gpu(v) for v in b]
    td = torch.float64 if dtype == np.float64 else torch.float32
    out_a = torch.empty(2, dtype=td, device="cuda")
    out_b = torch.empty(2, dtype=td, device="cuda")
    step("noalloc dot %s %s n=%d then n=%d" % (kind, np.dtype(dtype), n1, n2))
    # both calls enqueued back to back, the second reusing the array
    tf.tf_dot_noalloc(*ga, out_a)
    tf.tf_dot_noalloc(*gb, out_b)
    torch.cuda.synchronize()
    got_a, got_b = to_np(out_a), to_np(out_b)
    step("noalloc reference tf_dot %s %s" % (kind, np.dtype(dtype)))
    want_a = to_np(tf.tf_dot(*ga))
    want_b = to_np(tf.tf_dot(*gb))
    assert_bits(got_a, want_a, "first call n=%d" % n1)
    assert_bits(got_b, want_b, "second call n=%d" % n2)
    # and the workspace path itself against the oracle's tree
    assert_bits(want_b, np.array(oracle.dot(*b)), "tf_dot n=%d vs oracle" % n2)


@pytest.mark.parametrize("dtype", DTYPES)
def test_two_level_partials_then_small(dtype):
    """n past 2^28 leaves: the first pass leaves more than 65536 partials, so
    a middle level is stored in the array too; then a small call."""
    torch = torch_cuda()
    td = torch.float64 if dtype == np.float64 else torch.float32
    n1 = (1 << 28) + 12345
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    step("noalloc two-level n=%d %s: inputs" % (n1, np.dtype(dtype)))
    x0 = torch.randn(n1, dtype=td, device="cuda", generator=g)
    y0 = torch.randn(n1, dtype=td, device="cuda", generator=g)
    small = [to_gpu(v) for v in pick(random_case(1000, dtype, 9), "dd")]
    out1 = torch.empty(2, dtype=td, device="cuda")
    out2 = torch.empty(2, dtype=td, device="cuda")
    step("noalloc two-level n=%d %s: calls" % (n1, np.dtype(dtype)))
    tf.tf_dot_noalloc(x0, None, y0, None, out1)
    tf.tf_dot_noalloc(*small, out2)
    torch.cuda.synchronize()
    assert_bits(to_np(out1), to_np(tf.tf_dot(x0, None, y0, None)), "n=%d" % n1)
    assert_bits(to_np(out2), to_np(tf.tf_dot(*small)), "n=1000 after n=%d" % n1)
    del x0, y0
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", DTYPES)
def test_empty_writes_zero(dtype):
    torch = torch_cuda()
    td = torch.float64 if dtype == np.float64 else torch.float32
    e = torch.empty(0, dtype=td, device="cuda")
    out = torch.full((2,), 7.0, dtype=td, device="cuda")
    step("noalloc n=0 %s" % np.dtype(dtype))
    tf.tf_dot_noalloc(e, None, e, None, out)
    assert_bits(to_np(out), np.zeros(2, dtype=dtype), "n=0")


def test_tiling_adapts_then_rejects():
    """With one tile per block configured, 2^27 binary64 leaves would leave
    2^19 partials of 16 bytes (8 MiB): the call takes more tiles per block
    instead and still matches tf_dot bit for bit.  2^36 leaves leave too many
    partials even at 256 tiles per block: rejected on the host before any
    launch (the pointers are never read)."""
    torch = torch_cuda()
    lib = tf.lib()
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    big = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    big.fill_(0.5)
    big[1::3] = -0.25
    step("noalloc n=2^27 binary64 at one tile per block")
    old = tf.tf_config(tf.TF_CFG_RED_TILES_PER_BLOCK, 1)
    try:
        got = to_np(tf.tf_dot_noalloc(big, None, big, None, out))
        want = to_np(tf.tf_dot(big, None, big, None))
    finally:
        tf.tf_config(tf.TF_CFG_RED_TILES_PER_BLOCK, old)
    assert_bits(got, want, "n=2^27 at one tile per block")
    step("noalloc rejection of n=2^36")
    p = ctypes.c_void_p(big.data_ptr())
    st = lib.tf_dot_noalloc(tf.TF_F64, ctypes.c_int64(1 << 36), p, None, p, None,
                            ctypes.c_void_p(out.data_ptr()), None)
    assert st == -3  # TF_ENOMEM
    del big
    torch.cuda.empty_cache()
