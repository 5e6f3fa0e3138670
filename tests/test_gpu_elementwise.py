"""GPU parity: elementwise twofold operations, axpy, Horner and the plain
kernels, bit for bit against the oracle (NaN matched by class).

Sizes: the correctness configuration (n = 2^20, the paper-style operand
generator) plus ragged sizes that span several vector groups and leave a
tail, misaligned views (scalar path), special values, and sampled outputs
of the full-size axpy / Horner workloads (n = 2^28) in the launch
configuration the benchmark times.
"""
import numpy as np
import pytest

import oracle
import paper_1401_6235_amd as tf
from gpu_util import assert_bits, step, to_gpu, to_np, torch_cuda
from paper_1401_6235_amd import workloads as W

pytestmark = pytest.mark.gpu

DTYPES = [np.float64, np.float32]
OPS = ["add", "sub", "mul", "div"]
VARIANTS = [(True, True), (True, False), (False, True), (False, False)]


def _run_binary(op, c, xt, yt):
    x1 = c["x1"] if xt else None
    y1 = c["y1"] if yt else None
    want = getattr(oracle, op)(c["x0"], x1, c["y0"], y1)
    g = getattr(tf, "tf_" + op)(to_gpu(c["x0"]), to_gpu(x1), to_gpu(c["y0"]), to_gpu(y1))
    torch_cuda().cuda.synchronize()
    return (to_np(g[0]), to_np(g[1])), want


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", OPS)
def test_binary_config0(op, dtype):
    c = W.elementwise(op, 1 << 20, seed=0, dtype=dtype)
    for xt, yt in VARIANTS:
        step("binary %s %s xt=%d yt=%d n=2^20" % (op, np.dtype(dtype), xt, yt))
        got, want = _run_binary(op, c, xt, yt)
        assert_bits(got[0], want[0], "%s z0" % op)
        assert_bits(got[1], want[1], "%s z1" % op)


@pytest.mark.parametrize("dtype", DTYPES)
def test_sqrt_config0(dtype):
    c = W.elementwise("sqrt", 1 << 20, seed=0, dtype=dtype)
    for xt in (True, False):
        step("sqrt %s xt=%d n=2^20" % (np.dtype(dtype), xt))
        x1 = c["x1"] if xt else None
        want = oracle.sqrt(c["x0"], x1)
        g = tf.tf_sqrt(to_gpu(c["x0"]), to_gpu(x1))
        assert_bits(to_np(g[0]), want[0], "sqrt z0")
        assert_bits(to_np(g[1]), want[1], "sqrt z1")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 255, 257, 1023, 4099, 65537, 1000003])
def test_ragged_sizes(n, dtype):
    step("ragged n=%d %s" % (n, np.dtype(dtype)))
    for op in OPS:
        c = W.elementwise(op, n, seed=n, dtype=dtype)
        got, want = _run_binary(op, c, True, True)
        assert_bits(got[0], want[0], op)
        assert_bits(got[1], want[1], op)
    c = W.elementwise("sqrt", n, seed=n, dtype=dtype)
    g = tf.tf_sqrt(to_gpu(c["x0"]), to_gpu(c["x1"]))
    want = oracle.sqrt(c["x0"], c["x1"])
    assert_bits(to_np(g[0]), want[0], "sqrt")
    assert_bits(to_np(g[1]), want[1], "sqrt")


@pytest.mark.parametrize("dtype", DTYPES)
def test_misaligned_views_take_the_scalar_path(dtype):
    torch = torch_cuda()
    n = 100003
    c = W.elementwise("add", n + 1, seed=5, dtype=dtype)
    step("misaligned add %s" % np.dtype(dtype))
    base = {k: to_gpu(v) for k, v in c.items()}
    views = {k: v[1:] for k, v in base.items()}  # offset by one element
    z0 = torch.empty(n + 1, dtype=base["x0"].dtype, device="cuda")[1:]
    z1 = torch.empty(n + 1, dtype=base["x0"].dtype, device="cuda")[1:]
    tf.tf_add(views["x0"], views["x1"], views["y0"], views["y1"], z0, z1)
    want = oracle.add(c["x0"][1:], c["x1"][1:], c["y0"][1:], c["y1"][1:])
    assert_bits(to_np(z0), want[0], "z0")
    assert_bits(to_np(z1), want[1], "z1")


def special_values(dtype):
    t = np.dtype(dtype).type
    fi = np.finfo(dtype)
    vals = [0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, np.nan, fi.max, -fi.max, fi.tiny, -fi.tiny,
            fi.tiny * fi.eps, -fi.tiny * fi.eps, fi.eps, 3.0, 0.1, 1e-3, fi.tiny * 3.5]
    return np.array(vals, dtype=dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_special_values(dtype):
    """Signed zeros, infinities, NaN, subnormals and extremes in every
    position of every operation and variant."""
    v = special_values(dtype)
    m = v.size
    # all combinations of (x0, x1, y0, y1) drawn from the specials
    idx = np.indices((m, m, m, m)).reshape(4, -1)
    x0, x1, y0, y1 = (v[i] for i in idx)
    step("specials %s n=%d" % (np.dtype(dtype), x0.size))
    for op in OPS:
        for xt, yt in VARIANTS:
            c = {"x0": x0, "x1": x1, "y0": y0, "y1": y1}
            got, want = _run_binary(op, c, xt, yt)
            assert_bits(got[0], want[0], "%s z0 %d%d" % (op, xt, yt))
            assert_bits(got[1], want[1], "%s z1 %d%d" % (op, xt, yt))
    for xt in (True, False):
        a1 = x1 if xt else None
        g = tf.tf_sqrt(to_gpu(x0), to_gpu(a1))
        want = oracle.sqrt(x0, a1)
        assert_bits(to_np(g[0]), want[0], "sqrt z0")
        assert_bits(to_np(g[1]), want[1], "sqrt z1")


@pytest.mark.parametrize("dtype", DTYPES)
def test_division_and_sqrt_are_correctly_rounded(dtype):
    """The device's IEEE division and square root agree with the host's
    correctly rounded ones on many random operands (the plain kernels)."""
    g = np.random.default_rng(12)
    n = 1 << 22
    bits = g.integers(0, 2 ** 63 if dtype == np.float64 else 2 ** 31, (2, n), dtype=np.int64)
    if dtype == np.float64:
        a, b = bits.astype(np.uint64).view(np.float64)
    else:
        a, b = bits.astype(np.uint32).view(np.float32)
    step("div/sqrt rounding %s" % np.dtype(dtype))
    assert_bits(to_np(tf.tf_plain_div(to_gpu(a), to_gpu(b))), oracle.plain("div", a, b), "div")
    assert_bits(to_np(tf.tf_plain_sqrt(to_gpu(np.abs(a)))), oracle.plain("sqrt", np.abs(a)), "sqrt")
    z = tf.tf_mul(to_gpu(a), None, to_gpu(b), None)
    want = oracle.mul(a, None, b, None)
    assert_bits(to_np(z[1]), want[1], "fma error term")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 7, 4099, 1 << 20])
def test_axpy_and_horner(n, dtype):
    step("axpy/horner n=%d %s" % (n, np.dtype(dtype)))
    c = W.axpy_case(n, seed=1, dtype=dtype)
    for xt, yt in VARIANTS:
        x1 = c["x1"] if xt else None
        y1 = c["y1"] if yt else None
        want = oracle.axpy(c["a"], c["x0"], x1, c["y0"], y1)
        g = tf.tf_axpy(c["a"], to_gpu(c["x0"]), to_gpu(x1), to_gpu(c["y0"]), to_gpu(y1))
        assert_bits(to_np(g[0]), want[0], "axpy z0")
        assert_bits(to_np(g[1]), want[1], "axpy z1")
    h = W.horner_case(n, seed=1, dtype=dtype)
    for xt in (True, False):
        x1 = h["x1"] if xt else None
        want = oracle.horner(h["c"], h["x0"], x1)
        g = tf.tf_horner(h["c"], to_gpu(h["x0"]), to_gpu(x1))
        assert_bits(to_np(g[0]), want[0], "horner z0")
        assert_bits(to_np(g[1]), want[1], "horner z1")
    for deg in (0, 1, 3, 16, 32):
        cc = h["c"][: deg + 1] if deg <= 8 else np.resize(h["c"], deg + 1)
        want = oracle.horner(cc, h["x0"], h["x1"])
        g = tf.tf_horner(cc, to_gpu(h["x0"]), to_gpu(h["x1"]))
        assert_bits(to_np(g[0]), want[0], "horner deg %d z0" % deg)
        assert_bits(to_np(g[1]), want[1], "horner deg %d z1" % deg)


@pytest.mark.parametrize("dtype", DTYPES)
def test_plain_kernels(dtype):
    n = 100003
    c = W.elementwise("add", n, seed=2, dtype=dtype)
    x, y = c["x0"], c["y0"]
    gx, gy = to_gpu(x), to_gpu(y)
    step("plain kernels %s" % np.dtype(dtype))
    for op in OPS:
        assert_bits(to_np(getattr(tf, "tf_plain_" + op)(gx, gy)), oracle.plain(op, x, y), op)
    assert_bits(to_np(tf.tf_plain_sqrt(to_gpu(np.abs(x)))), oracle.plain("sqrt", np.abs(x)), "sqrt")
    assert_bits(to_np(tf.tf_vmem(gx, gy)), x, "vmem")
    a = W.axpy_case(n, seed=2, dtype=dtype)
    assert_bits(to_np(tf.tf_plain_axpy(a["a"][0], to_gpu(a["x0"]), to_gpu(a["y0"]))),
                oracle.plain_axpy(a["a"][0], a["x0"], a["y0"]), "plain axpy")
    h = W.horner_case(n, seed=2, dtype=dtype)
    assert_bits(to_np(tf.tf_plain_horner(h["c"], to_gpu(h["x0"]))), oracle.plain_horner(h["c"], h["x0"]),
                "plain horner")
    # the plain results are the twofold z0, bit for bit
    z = tf.tf_axpy(a["a"], to_gpu(a["x0"]), to_gpu(a["x1"]), to_gpu(a["y0"]), to_gpu(a["y1"]))
    assert_bits(to_np(z[0]), oracle.plain_axpy(a["a"][0], a["x0"], a["y0"]), "axpy z0 = plain")


def _f32_bounds(kind, case, idx, z0, z1, count):
    """binary32 z1 on `count` of the sampled elements against the binary64
    reference deviation of z0, within the running bound of the element's
    steps at u = 2^-24 plus the reference's own error (the same bound
    scaled to u = 2^-53, with a factor 2 to spare, and 2^-52 |dz0|)."""
    from exact import F
    from test_oracle_bounds import axpy_bound, horner_bound
    j = idx[:count]
    f32 = np.float32
    if kind == "axpy":
        dz = oracle.ref64("axpy", case["a"], case["x0"][j], case["x1"][j], case["y0"][j], case["y1"][j], z0[:count])
    else:
        dz = oracle.ref64("horner", case["c"], case["x0"][j], case["x1"][j], z0[:count])
    for k, i in enumerate(j):
        if kind == "axpy":
            b, exact = axpy_bound(case["a"], case["x0"][i], case["x1"][i], case["y0"][i], case["y1"][i], z0[k], f32)
        else:
            b, exact = horner_bound(case["c"], case["x0"][i], case["x1"][i], z0[k], f32)
        slack = b / 2 ** 28 + abs(exact) / 2 ** 52
        assert abs(F(dz[k]) - exact) <= slack, (kind, i)
        assert abs(F(z1[k]) - F(dz[k])) <= b + 2 * slack, (kind, i)


@pytest.mark.parametrize("dtype", DTYPES)
def test_full_size_sampled(dtype):
    """The n = 2^28 axpy and Horner workloads in the benchmark's launch
    configuration; 200k sampled outputs checked one by one against the
    oracle.  binary32 z1 is also judged against the binary64 reference
    deviation on 2000 of them, within each element's running bound."""
    torch = torch_cuda()
    n = 1 << 28
    name = np.dtype(dtype).name
    g = np.random.default_rng(77)
    idx = np.unique(np.concatenate([g.integers(0, n, 200000), [0, 1, n - 2, n - 1]]))
    g.shuffle(idx)
    step("full-size axpy %s n=2^28 (generate)" % name)
    c = W.axpy_case(n, seed=0, dtype=dtype)
    gpu = {k: to_gpu(v) for k, v in c.items() if k != "a"}
    step("full-size axpy %s n=2^28 (run)" % name)
    z = tf.tf_axpy(c["a"], gpu["x0"], gpu["x1"], gpu["y0"], gpu["y1"])
    torch.cuda.synchronize()
    want = oracle.axpy(c["a"], c["x0"][idx], c["x1"][idx], c["y0"][idx], c["y1"][idx])
    ii = torch.from_numpy(idx).cuda()
    got = (to_np(z[0][ii]), to_np(z[1][ii]))
    assert_bits(got[0], want[0], "axpy z0")
    assert_bits(got[1], want[1], "axpy z1")
    if dtype == np.float32:
        _f32_bounds("axpy", c, idx, got[0], got[1], 2000)
    del gpu, z, c
    torch.cuda.empty_cache()
    step("full-size horner %s n=2^28" % name)
    h = W.horner_case(n, seed=0, dtype=dtype)
    z = tf.tf_horner(h["c"], to_gpu(h["x0"]), to_gpu(h["x1"]))
    torch.cuda.synchronize()
    want = oracle.horner(h["c"], h["x0"][idx], h["x1"][idx])
    got = (to_np(z[0][ii]), to_np(z[1][ii]))
    assert_bits(got[0], want[0], "horner z0")
    assert_bits(got[1], want[1], "horner z1")
    if dtype == np.float32:
        _f32_bounds("horner", h, idx, got[0], got[1], 2000)
    del z, h
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", DTYPES)
def test_full_size_binary_ops_sampled(dtype):
    """The benchmark step's twofold add, sub, mul, div and sqrt at n = 2^28
    in its launch configuration, both operands twofold.  Inputs are seeded
    on the device (torch's generator: sign-uniform high parts of magnitude
    in [0.5, 1.5) times a power of two in 2^-20 .. 2^20, low parts about
    one unit in the last place of them; positive for the square root);
    100k sampled outputs, the first and last ones among them, are checked
    one by one against the oracle."""
    torch = torch_cuda()
    n = 1 << 28
    dt = torch.float32 if dtype == np.float32 else torch.float64
    ulp = 2.0 ** -24 if dtype == np.float32 else 2.0 ** -53
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2028)

    def hi(positive=False):
        v = (torch.rand(n, generator=gen, device="cuda", dtype=dt) + 0.5)
        v = v * torch.exp2(torch.randint(-20, 21, (n,), generator=gen, device="cuda").to(dt))
        if positive:
            return v
        sign = torch.randint(0, 2, (n,), generator=gen, device="cuda", dtype=torch.int8)
        return torch.where(sign == 1, -v, v)

    def lo(h):
        return h * ((torch.rand(n, generator=gen, device="cuda", dtype=dt) * 2 - 1) * ulp)

    g = np.random.default_rng(29)
    idx = np.unique(np.concatenate([g.integers(0, n, 100000), [0, 1, n - 2, n - 1]]))
    ii = torch.from_numpy(idx).cuda()
    name = np.dtype(dtype).name
    step("full-size binary ops %s n=2^28 (generate)" % name)
    x0 = hi()
    x1 = lo(x0)
    y0 = hi()
    y1 = lo(y0)
    z0, z1 = torch.empty_like(x0), torch.empty_like(x0)
    hx = [t.index_select(0, ii).cpu().numpy() for t in (x0, x1, y0, y1)]
    for op in ("add", "sub", "mul", "div"):
        step("full-size %s %s n=2^28" % (op, name))
        getattr(tf, "tf_" + op)(x0, x1, y0, y1, z0, z1)
        torch.cuda.synchronize()
        want = getattr(oracle, op)(*hx)
        assert_bits(to_np(z0.index_select(0, ii)), want[0], "%s z0" % op)
        assert_bits(to_np(z1.index_select(0, ii)), want[1], "%s z1" % op)
    del y0, y1
    step("full-size sqrt %s n=2^28" % name)
    s0 = hi(positive=True)
    s1 = lo(s0)
    tf.tf_sqrt(s0, s1, z0, z1)
    torch.cuda.synchronize()
    want = oracle.sqrt(s0.index_select(0, ii).cpu().numpy(), s1.index_select(0, ii).cpu().numpy())
    assert_bits(to_np(z0.index_select(0, ii)), want[0], "sqrt z0")
    assert_bits(to_np(z1.index_select(0, ii)), want[1], "sqrt z1")
    del x0, x1, s0, s1, z0, z1
    torch.cuda.empty_cache()


def test_repeat_and_grid_cap_are_bitwise_stable():
    torch = torch_cuda()
    c = W.elementwise("div", 1 << 20, seed=3)
    args = [to_gpu(c[k]) for k in ("x0", "x1", "y0", "y1")]
    step("grid cap determinism")
    a = [to_np(t) for t in tf.tf_div(*args)]
    old = tf.tf_config(tf.TF_CFG_EW_BLOCKS_PER_CU, 1)
    try:
        b = [to_np(t) for t in tf.tf_div(*args)]
    finally:
        tf.tf_config(tf.TF_CFG_EW_BLOCKS_PER_CU, old)
    torch.cuda.synchronize()
    assert_bits(a[0], b[0], "z0")
    assert_bits(a[1], b[1], "z1")
