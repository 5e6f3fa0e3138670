"""GPU parity: coupled (p) operations, Dekker mode, Fast Two-Sum
renormalisation and the in-register chains, bit for bit against the oracle
(NaN matched by class).

Sizes: n = 2^20 operands of the elementwise generator plus ragged sizes
around the vector groups; chains of 37 steps on ragged sizes around the
256 x 4 elements one block carries; the paper's two long-running examples
(the renormalisation count of ones and the clock accumulator) at their
full step counts; and sampled outputs of the chain workload the benchmark
times.
"""
import numpy as np
import pytest

import oracle
import paper_1401_6235_amd as tf
from gpu_util import assert_bits, step, to_gpu, to_np, torch_cuda
from paper_1401_6235_amd import workloads as W

pytestmark = pytest.mark.gpu

DTYPES = [np.float64, np.float32]
OPS = ["add", "sub", "mul", "div", "sqrt"]
MODES = ["twofold", "coupled", "dekker"]


def _coupled_both(op, c, xt, yt, renorm):
    x1 = c["x1"] if xt else None
    y0 = c.get("y0")
    y1 = c["y1"] if yt and op != "sqrt" else None
    want = oracle.coupled(op, c["x0"], x1, y0, y1, renorm=renorm)
    got = tf.tf_coupled(op, to_gpu(c["x0"]), to_gpu(x1), to_gpu(y0), to_gpu(y1), renorm=renorm)
    torch_cuda().cuda.synchronize()
    return (to_np(got[0]), to_np(got[1])), want


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("renorm", [False, True])
def test_coupled_operations(op, renorm, dtype):
    c = W.elementwise(op, 1 << 20, seed=3, dtype=dtype)
    forms = [(True, False), (False, False)] if op == "sqrt" else [(1, 1), (1, 0), (0, 1), (0, 0)]
    for xt, yt in forms:
        step("coupled %s renorm=%d %s xt=%d yt=%d n=2^20" % (op, renorm, np.dtype(dtype), xt, yt))
        got, want = _coupled_both(op, c, xt, yt, renorm)
        assert_bits(got[0], want[0], "%s z0" % op)
        assert_bits(got[1], want[1], "%s z1" % op)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 3, 257, 4099, 1000003])
def test_coupled_ragged(n, dtype):
    for op in OPS:
        step("coupled ragged %s n=%d %s" % (op, n, np.dtype(dtype)))
        c = W.elementwise(op, n, seed=n, dtype=dtype)
        got, want = _coupled_both(op, c, True, True, True)
        assert_bits(got[0], want[0], op)
        assert_bits(got[1], want[1], op)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [5, 1 << 20])
def test_renorm(n, dtype):
    c = W.elementwise("mul", n, seed=11, dtype=dtype)
    # pairs of every balance: coupled (x), loose and reversed (z1 >= z0)
    z0 = np.concatenate([c["x0"], c["x0"], c["y1"]])
    z1 = np.concatenate([c["x1"], c["y0"] * dtype(2.0 ** -10), c["y0"]])
    step("renorm n=%d %s" % (z0.size, np.dtype(dtype)))
    want = oracle.renorm(z0, z1)
    got = tf.tf_renorm(to_gpu(z0), to_gpu(z1))
    assert_bits(to_np(got[0]), want[0], "s")
    assert_bits(to_np(got[1]), want[1], "t")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", OPS)
def test_chains(op, dtype):
    for n in (1, 1023, 1025, 4099):
        c = W.chain_case(op, n, seed=n, dtype=dtype)
        for mode in MODES:
            for xt, yt in ((True, True), (False, False), (True, False)):
                step("chain %s %s %s n=%d xt=%d yt=%d reps=37" % (op, mode, np.dtype(dtype), n, xt, yt))
                x1 = c["x1"] if xt else None
                y0 = c.get("y0")
                y1 = c["y1"] if yt and op != "sqrt" else None
                want = oracle.chain(op, mode, 37, c["x0"], x1, y0, y1)
                got = tf.tf_chain(op, mode, 37, to_gpu(c["x0"]), to_gpu(x1), to_gpu(y0), to_gpu(y1))
                assert_bits(to_np(got[0]), want[0], "chain z0")
                assert_bits(to_np(got[1]), want[1], "chain z1")
        step("plain chain %s %s n=%d" % (op, np.dtype(dtype), n))
        want = oracle.plain_chain(op, 37, c["x0"], c.get("y0"))
        got = tf.tf_plain_chain(op, 37, to_gpu(c["x0"]), to_gpu(c.get("y0")))
        assert_bits(to_np(got), want, "plain chain")


@pytest.mark.parametrize("dtype", DTYPES)
def test_zero_step_chain(dtype):
    c = W.chain_case("mul", 3000, seed=1, dtype=dtype)
    step("chain reps=0 %s" % np.dtype(dtype))
    got = tf.tf_chain("mul", "twofold", 0, to_gpu(c["x0"]), to_gpu(c["x1"]), to_gpu(c["y0"]), to_gpu(c["y1"]))
    assert_bits(to_np(got[0]), c["x0"], "z0")
    assert_bits(to_np(got[1]), c["x1"], "z1")


def test_counting_ones_example():
    """The paper's renormalisation example in binary32: 2^25 + 2^20
    additions of 1 saturate a twofold at (2^24, 2^24) and count exactly in
    Dekker mode."""
    f32 = np.float32
    steps = 2 ** 25 + 2 ** 20
    n = 512
    x0, ones = np.zeros(n, f32), np.ones(n, f32)
    step("counting ones twofold reps=%d" % steps)
    z = tf.tf_chain("add", "twofold", steps, to_gpu(x0), None, to_gpu(ones), None)
    assert (to_np(z[0]) == 2.0 ** 24).all() and (to_np(z[1]) == 2.0 ** 24).all()
    step("counting ones dekker reps=%d" % steps)
    z = tf.tf_chain("add", "dekker", steps, to_gpu(x0), None, to_gpu(ones), None)
    s = to_np(z[0]).astype(np.float64) + to_np(z[1]).astype(np.float64)
    assert (s == steps).all() and (to_np(z[1]) == 0).all()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("hours", [100, 1000])
def test_clock_accumulator(hours, dtype):
    """The Applications section's clock: add the twofold 1/10 s 36000 times
    per hour, on many lanes at once (every lane equal to the oracle's
    sequential accumulator, bit for bit)."""
    t0 = np.asarray(0.1, dtype)
    t1 = np.asarray(np.float64(0.1) - np.float64(t0), dtype)
    steps = hours * 36000
    n = 256
    step("clock %dh %s reps=%d" % (hours, np.dtype(dtype), steps))
    z = tf.tf_chain("add", "twofold", steps, to_gpu(np.zeros(n, dtype)), to_gpu(np.zeros(n, dtype)),
                    to_gpu(np.full(n, t0, dtype)), to_gpu(np.full(n, t1, dtype)))
    s0, s1 = oracle.accumulate(steps, t0, t1)
    assert_bits(to_np(z[0]), np.full(n, s0, dtype), "clock z0")
    assert_bits(to_np(z[1]), np.full(n, s1, dtype), "clock z1")


CHAIN_N = 1 << 21
CHAIN_REPS = 2048


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", OPS)
def test_benchmark_chain_sampled(op, dtype):
    """The chain workload the benchmark times (n = 2^21, 2048 steps), with
    2048 sampled elements recomputed by the oracle."""
    c = W.chain_case(op, CHAIN_N, seed=0, dtype=dtype)
    idx = np.sort(np.random.default_rng(5).choice(CHAIN_N, 2048, replace=False))
    for mode in MODES:
        step("bench chain %s %s %s" % (op, mode, np.dtype(dtype)))
        got = tf.tf_chain(op, mode, CHAIN_REPS, to_gpu(c["x0"]), to_gpu(c["x1"]), to_gpu(c.get("y0")),
                          to_gpu(c.get("y1")))
        sub = {k: v[idx] for k, v in c.items()}
        want = oracle.chain(op, mode, CHAIN_REPS, sub["x0"], sub["x1"], sub.get("y0"), sub.get("y1"))
        assert_bits(to_np(got[0])[idx], want[0], "z0")
        assert_bits(to_np(got[1])[idx], want[1], "z1")


@pytest.mark.parametrize("dtype", DTYPES)
def test_special_values_coupled_and_renorm(dtype):
    """Signed zeros, infinities, NaN, subnormals and extremes in every
    position of the coupled and Dekker operations and of Fast Two-Sum."""
    from test_gpu_elementwise import special_values
    v = special_values(dtype)
    m = v.size
    idx = np.indices((m, m, m, m)).reshape(4, -1)
    c = dict(zip(("x0", "x1", "y0", "y1"), (v[i] for i in idx)))
    step("specials coupled %s n=%d" % (np.dtype(dtype), c["x0"].size))
    for op in OPS:
        forms = [(True, False), (False, False)] if op == "sqrt" else [(1, 1), (1, 0), (0, 1), (0, 0)]
        for renorm in (False, True):
            for xt, yt in forms:
                got, want = _coupled_both(op, c, xt, yt, renorm)
                assert_bits(got[0], want[0], "%s z0 %d%d r%d" % (op, xt, yt, renorm))
                assert_bits(got[1], want[1], "%s z1 %d%d r%d" % (op, xt, yt, renorm))
    got = tf.tf_renorm(to_gpu(c["x0"]), to_gpu(c["x1"]))
    want = oracle.renorm(c["x0"], c["x1"])
    assert_bits(to_np(got[0]), want[0], "renorm s")
    assert_bits(to_np(got[1]), want[1], "renorm t")


@pytest.mark.parametrize("dtype", DTYPES)
def test_special_values_chains(dtype):
    """Specials as start values and operands of short chains (NaN and
    infinities flow through every step as the oracle's do)."""
    from test_gpu_elementwise import special_values
    v = special_values(dtype)
    m = v.size
    idx = np.indices((m, m, m, m)).reshape(4, -1)
    x0, x1, y0, y1 = (v[i] for i in idx)
    for op in OPS:
        for mode in MODES:
            step("specials chain %s %s %s" % (op, mode, np.dtype(dtype)))
            want = oracle.chain(op, mode, 5, x0, x1, y0, y1)
            got = tf.tf_chain(op, mode, 5, to_gpu(x0), to_gpu(x1), to_gpu(y0), to_gpu(y1))
            assert_bits(to_np(got[0]), want[0], "chain z0")
            assert_bits(to_np(got[1]), want[1], "chain z1")
