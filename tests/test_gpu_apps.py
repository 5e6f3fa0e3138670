"""GPU parity: the batched applications (back-substitution, quadratic) and
the twofold fma, bit for bit against the oracle (NaN matched by class); the
plain counterparts against the oracle's main parts (z0 is the standard
result by definition).

Sizes: ragged batch counts around the 256-thread block, every system order
from 1 to the largest, the paper's Jordan blocks, the full-size batches the
benchmark times (sampled), misaligned fma operands (scalar path), and
strictly-lower matrix entries poisoned with NaN (never read).
"""
import numpy as np
import pytest

import oracle
import paper_1401_6235_amd as tf
from gpu_util import assert_bits, step, to_gpu, to_np, torch_cuda
from paper_1401_6235_amd import workloads as W

pytestmark = pytest.mark.gpu

DTYPES = [np.float64, np.float32]


def _poison_lower(U, m, nsys):
    U = U.reshape(m, m, nsys).copy()
    for i in range(m):
        U[i, :i] = np.nan
    return U.reshape(-1)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", ["jordan", "dense"])
@pytest.mark.parametrize("m", [1, 2, 3, 8, 16, 17, 64])
def test_trsv(m, kind, dtype):
    for nsys in (1, 255, 1000):
        c = W.trsv_case(m, nsys, seed=m + nsys, dtype=dtype, kind=kind)
        U0 = _poison_lower(c["U0"], m, nsys)
        U1 = _poison_lower(c["U1"], m, nsys)
        for ut, ft in ((True, True), (False, True), (True, False), (False, False)):
            step("trsv %s m=%d nsys=%d %s ut=%d ft=%d" % (kind, m, nsys, np.dtype(dtype), ut, ft))
            u1 = U1 if ut else None
            f1 = c["f1"] if ft else None
            want = oracle.trsv_upper(m, U0, u1, c["f0"], f1)
            got = tf.tf_trsv_upper(m, to_gpu(U0), to_gpu(u1), to_gpu(c["f0"]), to_gpu(f1))
            assert_bits(to_np(got[0]), want[0], "x0")
            assert_bits(to_np(got[1]), want[1], "x1")
        step("plain trsv %s m=%d nsys=%d" % (kind, m, nsys))
        got = tf.tf_plain_trsv_upper(m, to_gpu(U0), to_gpu(c["f0"]))
        want = oracle.trsv_upper(m, U0, U1, c["f0"], None)
        assert_bits(to_np(got), want[0], "plain x")


def test_trsv_paper_jordan_blocks():
    """The paper's four 3x3 runs, batched per working type, against the
    oracle (which reproduces the printed logs)."""
    from test_oracle_apps import jordan_batch
    from test_oracle_paper import LOGS, TYPES
    for type_name in ("float", "double"):
        dt = TYPES[type_name]
        runs = [r for r in LOGS["gauss"]["runs"] if r["type"] == type_name]
        U0, U1, f0 = jordan_batch(runs, dt)
        step("trsv paper jordan %s" % type_name)
        want = oracle.trsv_upper(3, U0, U1, f0, np.zeros_like(f0))
        got = tf.tf_trsv_upper(3, to_gpu(U0), to_gpu(U1), to_gpu(f0), to_gpu(np.zeros_like(f0)))
        assert_bits(to_np(got[0]), want[0], "x0")
        assert_bits(to_np(got[1]), want[1], "x1")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 7, 255, 4099, 1 << 20])
def test_quadratic(n, dtype):
    c = W.quadratic_case(n, seed=n, dtype=dtype)
    args = [c[k] for k in ("a0", "a1", "b0", "b1", "c0", "c1")]
    step("quadratic n=%d %s" % (n, np.dtype(dtype)))
    want = oracle.quadratic(*args)
    got = tf.tf_quadratic(*[to_gpu(a) for a in args])
    for g, w, name in zip(got, want, ("r0", "r1", "s0", "s1")):
        assert_bits(to_np(g), w, name)
    step("plain quadratic n=%d %s" % (n, np.dtype(dtype)))
    r, s = tf.tf_plain_quadratic(to_gpu(c["a0"]), to_gpu(c["b0"]), to_gpu(c["c0"]))
    assert_bits(to_np(r), want[0], "plain r")
    assert_bits(to_np(s), want[2], "plain s")


def test_quadratic_paper_rows():
    """a = 1, b = 2 and the paper's c values, on the GPU, against the oracle
    (which reproduces the printed float rows and the NaN flow)."""
    for dt in DTYPES:
        c64 = np.array([1e-8, 1 + 1e-8])
        c0 = c64.astype(dt)
        c1 = (c64 - c0.astype(np.float64)).astype(dt)
        a0, b0, z = np.ones(2, dt), np.full(2, 2, dt), np.zeros(2, dt)
        step("quadratic paper rows %s" % np.dtype(dt))
        want = oracle.quadratic(a0, z, b0, z, c0, c1)
        got = tf.tf_quadratic(*[to_gpu(v) for v in (a0, z, b0, z, c0, c1)])
        for g, w in zip(got, want):
            assert_bits(to_np(g), w, "paper row")


@pytest.mark.parametrize("dtype", DTYPES)
def test_quadratic_misaligned(dtype):
    torch = torch_cuda()
    n = 100003
    c = W.quadratic_case(n + 1, seed=12, dtype=dtype)
    keys = ("a0", "a1", "b0", "b1", "c0", "c1")
    step("quadratic misaligned %s" % np.dtype(dtype))
    views = [to_gpu(c[k])[1:] for k in keys]
    outs = tuple(torch.empty(n + 1, dtype=views[0].dtype, device="cuda")[1:] for _ in range(4))
    tf.tf_quadratic(*views, out=outs)
    want = oracle.quadratic(*[c[k][1:] for k in keys])
    for g, w in zip(outs, want):
        assert_bits(to_np(g), w, "misaligned quadratic")


FORMS = [(x, y, w) for x in (True, False) for y in (True, False) for w in (True, False)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 3, 1023, 65537, 1 << 20])
def test_fma(n, dtype):
    c = W.fma_case(n, seed=n, dtype=dtype)
    for xt, yt, wt in FORMS:
        step("fma n=%d %s forms=%d%d%d" % (n, np.dtype(dtype), xt, yt, wt))
        x1, y1, w1 = (c["x1"] if xt else None), (c["y1"] if yt else None), (c["w1"] if wt else None)
        want = oracle.fma(c["x0"], x1, c["y0"], y1, c["w0"], w1)
        got = tf.tf_fma(to_gpu(c["x0"]), to_gpu(x1), to_gpu(c["y0"]), to_gpu(y1), to_gpu(c["w0"]), to_gpu(w1))
        assert_bits(to_np(got[0]), want[0], "fma z0")
        assert_bits(to_np(got[1]), want[1], "fma z1")
    step("plain fma n=%d %s" % (n, np.dtype(dtype)))
    got = tf.tf_plain_fma(to_gpu(c["x0"]), to_gpu(c["y0"]), to_gpu(c["w0"]))
    assert_bits(to_np(got), oracle.plain_fma(c["x0"], c["y0"], c["w0"]), "plain fma")


@pytest.mark.parametrize("dtype", DTYPES)
def test_fma_misaligned(dtype):
    torch = torch_cuda()
    n = 100003
    c = W.fma_case(n + 1, seed=9, dtype=dtype)
    step("fma misaligned %s" % np.dtype(dtype))
    views = {k: to_gpu(v)[1:] for k, v in c.items()}
    z0 = torch.empty(n + 1, dtype=views["x0"].dtype, device="cuda")[1:]
    z1 = torch.empty(n + 1, dtype=views["x0"].dtype, device="cuda")[1:]
    tf.tf_fma(views["x0"], views["x1"], views["y0"], views["y1"], views["w0"], views["w1"], z0, z1)
    sub = {k: v[1:] for k, v in c.items()}
    want = oracle.fma(sub["x0"], sub["x1"], sub["y0"], sub["y1"], sub["w0"], sub["w1"])
    assert_bits(to_np(z0), want[0], "z0")
    assert_bits(to_np(z1), want[1], "z1")


TRSV_NSYS, TRSV_M = 1 << 20, 16
JORDAN_NSYS, JORDAN_M = 1 << 24, 3
QUAD_N = 1 << 24
FMA_N = 1 << 26


@pytest.mark.parametrize("dtype", DTYPES)
def test_benchmark_sizes_sampled(dtype):
    """The batches the benchmark times, with sampled outputs recomputed by
    the oracle (systems, roots and fma elements drawn at random)."""
    g = np.random.default_rng(8)
    c = W.trsv_case(TRSV_M, TRSV_NSYS, seed=0, dtype=dtype, kind="dense")
    step("bench trsv %s nsys=%d m=%d" % (np.dtype(dtype), TRSV_NSYS, TRSV_M))
    got = tf.tf_trsv_upper(TRSV_M, to_gpu(c["U0"]), to_gpu(c["U1"]), to_gpu(c["f0"]), to_gpu(c["f1"]))
    ks = np.sort(g.choice(TRSV_NSYS, 512, replace=False))
    m = TRSV_M
    U0 = c["U0"].reshape(m, m, TRSV_NSYS)[:, :, ks].reshape(-1)
    U1 = c["U1"].reshape(m, m, TRSV_NSYS)[:, :, ks].reshape(-1)
    f0 = c["f0"].reshape(m, TRSV_NSYS)[:, ks].reshape(-1)
    f1 = c["f1"].reshape(m, TRSV_NSYS)[:, ks].reshape(-1)
    want = oracle.trsv_upper(m, U0, U1, f0, f1)
    assert_bits(to_np(got[0]).reshape(m, TRSV_NSYS)[:, ks].reshape(-1), want[0], "x0")
    assert_bits(to_np(got[1]).reshape(m, TRSV_NSYS)[:, ks].reshape(-1), want[1], "x1")
    del got, c

    m, ns = JORDAN_M, JORDAN_NSYS
    c = W.trsv_case(m, ns, seed=0, dtype=dtype, kind="jordan")
    step("bench jordan %s nsys=%d m=%d" % (np.dtype(dtype), ns, m))
    got = tf.tf_trsv_upper(m, to_gpu(c["U0"]), to_gpu(c["U1"]), to_gpu(c["f0"]), to_gpu(c["f1"]))
    ks = np.sort(g.choice(ns, 4096, replace=False))
    sub = [c[k].reshape(m, m, ns)[:, :, ks].reshape(-1) for k in ("U0", "U1")]
    fs = [c[k].reshape(m, ns)[:, ks].reshape(-1) for k in ("f0", "f1")]
    want = oracle.trsv_upper(m, sub[0], sub[1], fs[0], fs[1])
    assert_bits(to_np(got[0]).reshape(m, ns)[:, ks].reshape(-1), want[0], "jordan x0")
    assert_bits(to_np(got[1]).reshape(m, ns)[:, ks].reshape(-1), want[1], "jordan x1")
    del got, c

    q = W.quadratic_case(QUAD_N, seed=0, dtype=dtype)
    keys = ("a0", "a1", "b0", "b1", "c0", "c1")
    step("bench quadratic %s n=%d" % (np.dtype(dtype), QUAD_N))
    got = tf.tf_quadratic(*[to_gpu(q[k]) for k in keys])
    idx = np.sort(g.choice(QUAD_N, 1 << 14, replace=False))
    want = oracle.quadratic(*[q[k][idx] for k in keys])
    for gg, w in zip(got, want):
        assert_bits(to_np(gg)[idx], w, "quadratic")
    del got, q

    f = W.fma_case(FMA_N, seed=0, dtype=dtype)
    step("bench fma %s n=%d" % (np.dtype(dtype), FMA_N))
    got = tf.tf_fma(*[to_gpu(f[k]) for k in ("x0", "x1", "y0", "y1", "w0", "w1")])
    idx = np.sort(g.choice(FMA_N, 1 << 14, replace=False))
    want = oracle.fma(*[f[k][idx] for k in ("x0", "x1", "y0", "y1", "w0", "w1")])
    assert_bits(to_np(got[0])[idx], want[0], "fma z0")
    assert_bits(to_np(got[1])[idx], want[1], "fma z1")


@pytest.mark.parametrize("dtype", DTYPES)
def test_special_values_fma_and_quadratic(dtype):
    """Specials in every position of the fma (all operand forms) and of the
    quadratic's coefficients."""
    from test_gpu_elementwise import special_values
    v = special_values(dtype)
    m = v.size
    g = np.random.default_rng(4)
    idx = g.integers(0, m, (6, 1 << 18))
    x0, x1, y0, y1, w0, w1 = (v[i] for i in idx)
    for xt, yt, wt in FORMS:
        step("specials fma %s forms=%d%d%d" % (np.dtype(dtype), xt, yt, wt))
        a1, b1, c1 = (x1 if xt else None), (y1 if yt else None), (w1 if wt else None)
        want = oracle.fma(x0, a1, y0, b1, w0, c1)
        got = tf.tf_fma(to_gpu(x0), to_gpu(a1), to_gpu(y0), to_gpu(b1), to_gpu(w0), to_gpu(c1))
        assert_bits(to_np(got[0]), want[0], "fma z0")
        assert_bits(to_np(got[1]), want[1], "fma z1")
    step("specials quadratic %s" % np.dtype(dtype))
    want = oracle.quadratic(x0, x1, y0, y1, w0, w1)
    got = tf.tf_quadratic(*[to_gpu(a) for a in (x0, x1, y0, y1, w0, w1)])
    for gg, w in zip(got, want):
        assert_bits(to_np(gg), w, "quadratic")
