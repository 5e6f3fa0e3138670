"""Seeded synthetic inputs for the twofold hot path.

Both the GPU library's tests and benchmark and the oracle's tests draw their
inputs from here.  The module holds none of the twofold method's
arithmetic: only random draws (numpy PCG64 streams), assembly of binary64 /
binary32 values from random bits, one plain multiply that forms each
operand's low part, and (in ``illdot.c``) an exact-integer construction of
ill-conditioned dot products.

Every generator is a pure function of its arguments.  Streams are keyed by
``numpy.random.SeedSequence(seed, spawn_key=(purpose, ...))`` so each array
has its own stream and draw order inside a stream is stated per function.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TF_WORKLOADS_LIB selects another build of the library (the sanitizer tests use it)
LIB_PATH = os.environ.get("TF_WORKLOADS_LIB") or os.path.join(_HERE, "libtfgen.so")
SOURCE = os.path.join(_HERE, "illdot.c")

# Stream keys (first element of the spawn key).
_K_X, _K_Y, _K_AXPY, _K_HORNER, _K_DOT = 1, 2, 3, 4, 5
_K_CHAIN, _K_TRSV, _K_QUAD, _K_FMA = 7, 8, 9, 10

F64 = np.dtype(np.float64)
F32 = np.dtype(np.float32)


def build(force: bool = True) -> str:
    """Compile the exact ill-conditioned-dot generator with gcc."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", tmp, SOURCE, "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _gen_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        for name in ("tfgen_illdot_f64", "tfgen_illdot_f32", "tfgen_product_split_f64",
                     "tfgen_product_split_f32"):
            getattr(_lib, name).restype = None
        _lib.tfgen_exact_dot_f64.restype = C.c_double
    return _lib


def rng(seed: int, *key: int) -> np.random.Generator:
    """Independent PCG64 stream for (seed, key)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=tuple(key))))


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# Twofold operands: sign-uniform, mantissa uniform in [1, 2), exponent
# uniform in [exp_lo, exp_hi]; low part x1 = x0 * (u * 2^-p) with u uniform
# in [-1, 1) and p the precision (53 or 24).
# ---------------------------------------------------------------------------

def twofold_operand(n: int, seed: int, stream: int, dtype=F64, exp_lo: int = -20,
                    exp_hi: int = 20):
    """(x0, x1) for one operand.

    Draw order in stream (seed, stream): sign bits (n integers in {0, 1}),
    exponents (n integers in [exp_lo, exp_hi]), mantissa fractions (n
    integers in [0, 2^52) or [0, 2^23)), u (n doubles uniform in [-1, 1)).
    x0 is assembled bit by bit, so its mantissa is exactly 1 + k 2^-52
    (2^-23 for binary32).
    """
    dtype = np.dtype(dtype)
    g = rng(seed, stream)
    sign = g.integers(0, 2, n, dtype=np.uint64)
    expo = g.integers(exp_lo, exp_hi + 1, n, dtype=np.int64)
    if dtype == F64:
        frac = g.integers(0, 1 << 52, n, dtype=np.uint64)
        bits = (sign << np.uint64(63)) | ((expo + 1023).astype(np.uint64) << np.uint64(52)) | frac
        del sign, expo, frac
        x0 = bits.view(np.float64)
        u = g.uniform(-1.0, 1.0, n)
        u *= 2.0 ** -53
        x1 = x0 * u
    elif dtype == F32:
        frac = g.integers(0, 1 << 23, n, dtype=np.uint64)
        bits = ((sign << np.uint64(31)) | ((expo + 127).astype(np.uint64) << np.uint64(23)) | frac)
        del sign, expo, frac
        x0 = bits.astype(np.uint32).view(np.float32)
        u = g.uniform(-1.0, 1.0, n).astype(np.float32)
        u *= np.float32(2.0 ** -24)
        x1 = x0 * u
    else:
        raise TypeError(dtype)
    return np.ascontiguousarray(x0), x1


def elementwise(op: str, n: int, seed: int = 0, dtype=F64):
    """Operands of one elementwise call: dict with x0, x1, y0, y1.

    x comes from stream 1 and y from stream 2.  For sqrt the argument is
    made non-negative without changing its value's magnitude: x0 <- |x0|
    and x1 <- sign(x0) x1, i.e. the operand becomes |x|.  Divisors need no
    adjustment: |y0| >= 2^-20 already.
    """
    x0, x1 = twofold_operand(n, seed, _K_X, dtype)
    if op == "sqrt":
        neg = np.signbit(x0)
        x0 = np.abs(x0)
        x1 = np.where(neg, -x1, x1)
        return {"x0": x0, "x1": x1}
    y0, y1 = twofold_operand(n, seed, _K_Y, dtype)
    return {"x0": x0, "x1": x1, "y0": y0, "y1": y1}


AXPY_A = (0.7, 1e-17)


def axpy_case(n: int, seed: int = 0, dtype=F64):
    """a = (0.7, 1e-17) rounded to the working type; x, y twofold operands."""
    dtype = np.dtype(dtype)
    a = np.array(AXPY_A, dtype=dtype)
    x0, x1 = twofold_operand(n, seed, _K_AXPY, dtype)
    y0, y1 = twofold_operand(n, seed, _K_AXPY + 100, dtype)
    return {"a": a, "x0": x0, "x1": x1, "y0": y0, "y1": y1}


def horner_case(n: int, seed: int = 0, dtype=F64, degree: int = 8):
    """Coefficients c[0..degree] uniform in [-1, 1] with c[1] = 0; x0 uniform
    in [0.9, 1.1]; x1 = x0 * (u 2^-p).

    Draw order in stream (seed, 4): degree+1 coefficient doubles, then n
    doubles for x0, then n doubles for u.
    """
    dtype = np.dtype(dtype)
    g = rng(seed, _K_HORNER)
    c = g.uniform(-1.0, 1.0, degree + 1)
    if degree >= 1:
        c[1] = 0.0
    x0 = g.uniform(0.9, 1.1, n)
    u = g.uniform(-1.0, 1.0, n)
    if dtype == F64:
        u *= 2.0 ** -53
        x1 = x0 * u
        return {"c": c, "x0": x0, "x1": x1}
    c32 = c.astype(np.float32)
    x032 = x0.astype(np.float32)
    u32 = u.astype(np.float32) * np.float32(2.0 ** -24)
    return {"c": c32, "x0": x032, "x1": x032 * u32}


# ---------------------------------------------------------------------------
# Chains, batched applications, fma
# ---------------------------------------------------------------------------

def _low_part(x0, g, dtype):
    """x1 = x0 * (u 2^-p), u uniform in [-1, 1) (n doubles from g)."""
    u = g.uniform(-1.0, 1.0, x0.size)
    if np.dtype(dtype) == F64:
        return x0 * (u * 2.0 ** -53)
    return x0 * (u.astype(np.float32) * np.float32(2.0 ** -24))


def chain_case(op: str, n: int, seed: int = 0, dtype=F64):
    """Start values x and operands y for chains of many steps that stay in
    range: x a twofold operand with exponents in [-4, 4] (|x| for sqrt);
    for add / sub, y a twofold operand with exponents in [-16, -8]; for mul /
    div, y0 = 1 + v 2^-12 with v uniform in [-1, 1) (a few thousand steps
    change the value by a factor of at most e or so), y1 = y0 u 2^-p.

    Draw order: x from stream (seed, 7, 1); y from stream (seed, 7, 2): for
    mul / div n doubles v then n doubles u.
    """
    dtype = np.dtype(dtype)
    x0, x1 = twofold_operand(n, seed, _K_CHAIN, dtype, -4, 4)
    out = {"x0": x0, "x1": x1}
    if op == "sqrt":
        neg = np.signbit(x0)
        out["x0"] = np.abs(x0)
        out["x1"] = np.where(neg, -x1, x1)
        return out
    if op in ("add", "sub"):
        y0, y1 = twofold_operand(n, seed + 7919, _K_CHAIN, dtype, -16, -8)
    else:
        g = rng(seed, _K_CHAIN, 2)
        y0 = (1.0 + g.uniform(-1.0, 1.0, n) * 2.0 ** -12).astype(dtype)
        y1 = _low_part(y0, g, dtype)
    out.update(y0=np.ascontiguousarray(y0), y1=np.ascontiguousarray(y1))
    return out


def trsv_case(m: int, nsys: int, seed: int = 0, dtype=F64, kind: str = "jordan"):
    """Upper-triangular systems, interleaved (entry (i, j) of system k at
    [(i*m + j)*nsys + k], f_i at [i*nsys + k]); the strictly lower part is 0.

    kind "jordan" (the paper's test matrix): diagonal lambda_k with |lambda|
    log-uniform in [2^-min(10, 40/m), 1] and a random sign, 1 on the first
    superdiagonal; for binary32 lambda is drawn as a double and split into
    its float and the float of the remainder, as the paper initialises it.
    kind "dense": entries above the diagonal uniform in [-1, 1), diagonal
    +-(1 + uniform[0, 1)), low parts x0 u 2^-p.  f is a twofold operand with
    exponents in [-2, 2].  Growth stays below 2^64 in both kinds.

    Draw order in stream (seed, 8, m): jordan: nsys doubles for log2|lambda|,
    nsys sign integers; dense: m*m*nsys doubles for the entries, m*nsys
    doubles for the diagonal magnitudes, m*nsys sign integers, m*m*nsys
    doubles u for the low parts.
    """
    dtype = np.dtype(dtype)
    g = rng(seed, _K_TRSV, m)
    U0 = np.zeros((m, m, nsys), np.float64)
    U1 = np.zeros((m, m, nsys), np.float64)
    if kind == "jordan":
        lo = -min(10.0, 40.0 / m)
        lam = np.exp2(g.uniform(lo, 0.0, nsys)) * np.where(g.integers(0, 2, nsys) == 1, -1.0, 1.0)
        lam0 = lam.astype(dtype)
        lam1 = (lam - lam0.astype(np.float64)).astype(dtype)
        for i in range(m):
            U0[i, i] = lam0
            U1[i, i] = lam1
            if i + 1 < m:
                U0[i, i + 1] = 1.0
        U0, U1 = U0.astype(dtype), U1.astype(dtype)
    elif kind == "dense":
        vals = g.uniform(-1.0, 1.0, (m, m, nsys))
        diag = 1.0 + g.uniform(0.0, 1.0, (m, nsys))
        sgn = np.where(g.integers(0, 2, (m, nsys)) == 1, -1.0, 1.0)
        upper = np.triu(np.ones((m, m), bool), 1)[:, :, None]
        U0 = np.where(upper, vals, 0.0)
        for i in range(m):
            U0[i, i] = diag[i] * sgn[i]
        U0 = U0.astype(dtype)
        U1 = np.where(U0 != 0, _low_part(U0.reshape(-1), g, dtype).reshape(U0.shape), 0).astype(dtype)
    else:
        raise ValueError(kind)
    f0, f1 = twofold_operand(m * nsys, seed, _K_TRSV + 100 * m, dtype, -2, 2)
    return {"m": m, "U0": np.ascontiguousarray(U0.reshape(-1)), "U1": np.ascontiguousarray(U1.reshape(-1)),
            "f0": f0, "f1": f1}


def quadratic_case(n: int, seed: int = 0, dtype=F64):
    """Coefficients of a x^2 + b x + c with twofold parts: a, b twofold
    operands with exponents in [-2, 2]; c in three equal-odds classes:
    random (either sign of the discriminant), small (c = b^2 / (4a) times
    2^-k, k uniform in [20, 40]: the cancellation of the paper's c = 1e-8
    example) and near a double root (c = b^2 / (4a) (1 + v 2^-20), v
    uniform in [-1, 1)).  c1 = c0 u 2^-p.

    Draw order: a, b from streams (seed, 9, 1), (seed, 9, 2); stream
    (seed, 9, 3): n class integers, n doubles r (random class, c = r in
    [-4, 4)), n integers k, n doubles v, n doubles u.
    """
    dtype = np.dtype(dtype)
    a0, a1 = twofold_operand(n, seed, _K_QUAD, dtype, -2, 2)
    b0, b1 = twofold_operand(n, seed + 7919, _K_QUAD, dtype, -2, 2)
    g = rng(seed, _K_QUAD, 3)
    cls = g.integers(0, 3, n)
    r = g.uniform(-4.0, 4.0, n)
    k = g.integers(20, 41, n)
    v = g.uniform(-1.0, 1.0, n)
    crit = b0.astype(np.float64) ** 2 / (4.0 * a0.astype(np.float64))
    c = np.where(cls == 0, r, np.where(cls == 1, crit * np.exp2(-k.astype(np.float64)), crit * (1 + v * 2.0 ** -20)))
    c0 = c.astype(dtype)
    c1 = _low_part(c0, g, dtype)
    return {"a0": a0, "a1": a1, "b0": b0, "b1": b1, "c0": c0, "c1": np.ascontiguousarray(c1)}


def fma_case(n: int, seed: int = 0, dtype=F64):
    """x, y, w twofold operands with exponents in [-10, 10]; for one third of
    the elements w0 = -(x0 y0)(1 + v 2^-20), rounded (v uniform in [-1, 1)),
    so that the fma cancels.

    Draw order: x, y, w from streams (seed, 10, 1/2/3); stream (seed, 10, 4):
    n class integers then n doubles v.
    """
    dtype = np.dtype(dtype)
    x0, x1 = twofold_operand(n, seed, _K_FMA, dtype, -10, 10)
    y0, y1 = twofold_operand(n, seed + 7919, _K_FMA, dtype, -10, 10)
    w0, w1 = twofold_operand(n, seed + 15838, _K_FMA, dtype, -10, 10)
    g = rng(seed, _K_FMA, 4)
    near = g.integers(0, 3, n) == 0
    v = g.uniform(-1.0, 1.0, n)
    w0 = np.where(near, -(x0.astype(np.float64) * y0.astype(np.float64)) * (1 + v * 2.0 ** -20), w0).astype(dtype)
    return {"x0": x0, "x1": x1, "y0": y0, "y1": y1, "w0": np.ascontiguousarray(w0), "w1": w1}


# ---------------------------------------------------------------------------
# Ill-conditioned dot products (exact construction in illdot.c)
# ---------------------------------------------------------------------------

def _illdot_once(n, cond, e_max, seed, dtype):
    g = rng(seed, _K_DOT, int(round(math.log10(cond) * 100)), e_max)
    h = n // 2
    u = g.uniform(-1.0, 1.0, n)
    v = g.uniform(-1.0, 1.0, n)
    e1 = g.integers(0, e_max + 1, h, dtype=np.int64).astype(np.int32)
    if h >= 1:
        e1[0] = e_max
        e1[h - 1] = 0
    e1 = np.ascontiguousarray(e1)
    stats = np.zeros(3, np.float64)
    lib = _gen_lib()
    if dtype == F64:
        x, y = np.empty(n, np.float64), np.empty(n, np.float64)
        lib.tfgen_illdot_f64(C.c_int64(n), C.c_int(e_max), C.c_double(cond), _ptr(u), _ptr(v),
                             _ptr(e1), _ptr(x), _ptr(y), _ptr(stats))
    else:
        u32 = np.ascontiguousarray(u.astype(np.float32))
        v32 = np.ascontiguousarray(v.astype(np.float32))
        x, y = np.empty(n, np.float32), np.empty(n, np.float32)
        lib.tfgen_illdot_f32(C.c_int64(n), C.c_int(e_max), C.c_double(cond), _ptr(u32),
                             _ptr(v32), _ptr(e1), _ptr(x), _ptr(y), _ptr(stats))
    return x, y, {"cond": float(stats[0]), "dot": float(stats[1]), "e_max": e_max}


def illdot_case(n: int, cond: float, seed: int = 0, dtype=F64, max_tries: int = 8):
    """Dot instance (x, y) of length n (even) with condition number
    2 sum|x_i y_i| / |x^T y| close to ``cond``.

    First-half exponents are drawn uniformly in [0, e_max], starting from
    e_max = floor(log2(cond) / 2).  When the achieved condition number is
    more than a factor 4 away from the target, e_max moves by
    round(log2(ratio) / 2) and the instance is drawn again (the draws are
    keyed by e_max, so the result is a pure function of the arguments).
    Returns dict x, y, cond (achieved), dot (exact x^T y rounded once),
    e_max.
    """
    dtype = np.dtype(dtype)
    if n % 2:
        raise ValueError("illdot_case needs an even n")
    e_max = max(0, int(math.floor(math.log2(cond) / 2.0)))
    best = None
    for _ in range(max_tries):
        x, y, st = _illdot_once(n, cond, e_max, seed, dtype)
        ratio = st["cond"] / cond
        if best is None or abs(math.log(ratio)) < abs(math.log(best[2]["cond"] / cond)):
            best = (x, y, st)
        if 0.25 <= ratio <= 4.0:
            break
        step = int(round(math.log2(ratio) / 2.0)) or (1 if ratio > 1 else -1)
        new = max(0, e_max - step)
        if new == e_max:
            break
        e_max = new
    x, y, st = best
    return {"x": x, "y": y, "cond": st["cond"], "dot": st["dot"], "e_max": st["e_max"]}


def product_split(x, y):
    """(hi, lo) with hi = fl(x_i y_i) and lo = x_i y_i - hi exactly, from the
    exact integer product: twofold leaves whose sum is exactly x^T y."""
    dt = np.asarray(x).dtype
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y)
    hi, lo = np.empty_like(x), np.empty_like(x)
    fn = _gen_lib().tfgen_product_split_f64 if dt == F64 else _gen_lib().tfgen_product_split_f32
    fn(C.c_int64(x.size), _ptr(x), _ptr(y), _ptr(hi), _ptr(lo))
    return hi, lo


def sum_case(n: int, cond: float, seed: int = 0, dtype=F64):
    """Twofold sum instance: the exact product split of an ill-conditioned
    dot instance, so sum(x0_i + x1_i) = x^T y exactly."""
    d = illdot_case(n, cond, seed, dtype)
    x0, x1 = product_split(d["x"], d["y"])
    return {"x0": x0, "x1": x1, "cond": d["cond"], "dot": d["dot"], "e_max": d["e_max"]}


def exact_dot_f64(x, y) -> float:
    """Exact x^T y of binary64 vectors, rounded once (for reports)."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    return float(_gen_lib().tfgen_exact_dot_f64(C.c_int64(x.size), _ptr(x), _ptr(y)))


# ---------------------------------------------------------------------------
# Serving jobs: the counter-based generator the device uses for RANDOM and
# ILLCOND jobs, implemented again here from its published definition
# (SplitMix64: Steele, Lea and Flood 2014, with the finaliser constants of
# Vigna's splitmix64), so that a job's inputs can be rebuilt on the host
# bit for bit.  Element i of array a (0: x0, 1: x1, 2: y0, 3: y1) draws
# mix(seed + (4 i + a + 1) * gamma).
# ---------------------------------------------------------------------------

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def _mix64(z):
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
    return z ^ (z >> np.uint64(31))


def serve_draw(seed: int, n: int, a: int):
    i = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        k = i * np.uint64(4) + np.uint64(a + 1)
        return _mix64(np.uint64(seed) + k * _GAMMA)


def _serve_value(r, dtype):
    e = ((r >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) % 41 - 20
    if dtype == F64:
        bits = (r & np.uint64(0x8000000000000000)) | ((e + 1023).astype(np.uint64) << np.uint64(52)) \
            | (r & np.uint64(0xFFFFFFFFFFFFF))
        return bits.view(np.float64)
    bits = ((r >> np.uint64(32)) & np.uint64(0x80000000)) | ((e + 127).astype(np.uint64) << np.uint64(23)) \
        | (r & np.uint64(0x7FFFFF))
    return bits.astype(np.uint32).view(np.float32)


def _serve_u(r, dtype):
    if dtype == F64:
        return (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
    return (r >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -23) - np.float32(1.0)


def _serve_u01(r, dtype):
    if dtype == F64:
        return (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return (r >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)


def serve_inputs(op: str, dtype, n: int, seed: int, kind: str = "random", a0: float = 0.7):
    """Inputs of a RANDOM / ILLCOND serving job, as the device generates them.

    sum: twofold leaves (x0, x1); dot: plain x0, y0; axpy: twofold x, y
    (ILLCOND: y0 = -(a0 x0) + x0 (u 2^-40), 2^-16 in binary32, so that
    a x + y cancels); Horner: twofold x with x0 = 0.9 + 0.2 u01 (ILLCOND:
    x0 = 1 + u 2^-12).  Low parts are x1 = x0 (u 2^-p).
    """
    dtype = np.dtype(dtype)
    t = dtype.type
    low = t(2.0 ** -53) if dtype == F64 else t(2.0 ** -24)
    r0 = serve_draw(seed, n, 0)
    if op == "horner":
        if kind == "illcond":
            x0 = t(1) + _serve_u(r0, dtype) * t(2.0 ** -12)
        else:
            x0 = t(0.9) + t(0.2) * _serve_u01(r0, dtype)
    else:
        x0 = _serve_value(r0, dtype)
    out = {"x0": x0}
    if op in ("sum", "axpy", "horner"):
        out["x1"] = x0 * (_serve_u(serve_draw(seed, n, 1), dtype) * low)
    if op in ("dot", "axpy"):
        r2 = serve_draw(seed, n, 2)
        if op == "axpy" and kind == "illcond":
            cs = t(2.0 ** -40) if dtype == F64 else t(2.0 ** -16)
            a = t(a0)
            y0 = -(a * x0) + x0 * (_serve_u(r2, dtype) * cs)
        else:
            y0 = _serve_value(r2, dtype)
        out["y0"] = y0
        if op == "axpy":
            out["y1"] = y0 * (_serve_u(serve_draw(seed, n, 3), dtype) * low)
    return out


HORNER_ILLCOND_C = [1.0, -8.0, 28.0, -56.0, 70.0, -56.0, 28.0, -8.0, 1.0]  # (x - 1)^8


def serve_schedule(jobs: int, rate: float, seed: int = 1, min_log2: int = 8, max_log2: int = 24,
                   illcond_frac: float = 0.05):
    """The serving stream: Poisson arrivals at `rate` jobs/s; type uniform
    over sum / dot / axpy / Horner-8; length floor(2^(min + (max - min) U));
    binary32 or binary64 with probability 1/2; a fraction `illcond_frac`
    of ill-conditioned jobs.  Draw order in stream (seed, 6): gaps, types,
    dtypes, lengths, ill-conditioned marks, job seeds, Horner coefficient
    sets."""
    g = rng(seed, 6)
    gaps = g.exponential(1.0 / rate, jobs)
    types = g.integers(0, 4, jobs)
    dts = g.integers(0, 2, jobs)
    lens = np.floor(2.0 ** (min_log2 + (max_log2 - min_log2) * g.random(jobs))).astype(np.int64)
    ill = g.random(jobs) < illcond_frac
    seeds = g.integers(0, 2 ** 63, jobs, dtype=np.int64)
    coeffs = g.uniform(-1.0, 1.0, (jobs, 9))
    coeffs[:, 1] = 0.0
    names = ["sum", "dot", "axpy", "horner"]
    out = []
    t = 0.0
    for k in range(jobs):
        t += gaps[k]
        out.append({"t": t, "op": names[types[k]], "dtype": "f64" if dts[k] else "f32",
                    "n": int(lens[k]), "illcond": bool(ill[k]), "seed": int(seeds[k]),
                    "c": coeffs[k].tolist()})
    return out
