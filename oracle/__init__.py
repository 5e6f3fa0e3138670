"""Twofold-arithmetic oracle: a plain scalar C library loaded with ctypes.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_1401_6235_amd``) never imports, links or runs it, and the two share
no code: the only thing both sides use is the seeded input generators of
``paper_1401_6235_amd.workloads``, which hold none of the method's arithmetic.

Every function takes numpy arrays of float64 (the binary64 oracle) or
float32 (its binary32 mirror) and returns new numpy arrays.  A low part of
``None`` marks a dotted operand and selects the paper's *.1 / *.1.1
variants.  The C source (``tf_oracle.c``) documents which algorithm of the
paper each function follows.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TF_ORACLE_LIB selects another build of the library (the sanitizer tests use it)
LIB_PATH = os.environ.get("TF_ORACLE_LIB") or os.path.join(_HERE, "libtforacle.so")
SOURCES = [os.path.join(_HERE, "tf_oracle.c"), os.path.join(_HERE, "tf_oracle_t.h")]

# Contraction off and no fast-math: every a*b+c stays a multiply and an add.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libtforacle.so``."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, "-o", tmp, SOURCES[0], "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
    return _lib


@contextlib.contextmanager
def use_library(path: str):
    """Temporarily route every function here through another build of the
    oracle (used by the tests that plant mistakes in a copy of it)."""
    global _lib
    old = _lib
    _lib = C.CDLL(path)
    try:
        yield
    finally:
        _lib = old


_SFX = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}


def _sfx(a) -> str:
    dt = np.asarray(a).dtype
    if dt not in _SFX:
        raise TypeError("oracle takes float64 or float32 arrays, got %s" % dt)
    return _SFX[dt]


def _p(a):
    """Pointer to a contiguous array, or NULL for None."""
    if a is None:
        return None
    return a.ctypes.data_as(C.c_void_p)


def _arr(a, dt):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=dt)


def _fn(name: str):
    f = getattr(lib(), name)
    f.restype = None
    return f


def _binary(op: str, x0, x1, y0, y1):
    dt = np.asarray(x0).dtype
    x0, x1, y0, y1 = (_arr(v, dt) for v in (x0, x1, y0, y1))
    n = x0.size
    z0 = np.empty(n, dt)
    z1 = np.empty(n, dt)
    _fn("orc_%s_%s" % (op, _sfx(x0)))(C.c_int64(n), _p(x0), _p(x1), _p(y0), _p(y1), _p(z0), _p(z1))
    return z0, z1


def add(x0, x1, y0, y1):
    """ATF1 (ATF1.1 / Two-Sum when operands are dotted)."""
    return _binary("add", x0, x1, y0, y1)


def sub(x0, x1, y0, y1):
    """STF1 (STF1.1 / Two-Diff when operands are dotted)."""
    return _binary("sub", x0, x1, y0, y1)


def mul(x0, x1, y0, y1):
    """MTF1 (MTF1.1 / Two-Product when operands are dotted)."""
    return _binary("mul", x0, x1, y0, y1)


def div(x0, x1, y0, y1):
    """DTF1 (DTF1.1 / DTF1.1.1 when operands are dotted)."""
    return _binary("div", x0, x1, y0, y1)


def sqrt(x0, x1):
    """RTF1 (RPF1.1 when the argument is dotted)."""
    dt = np.asarray(x0).dtype
    x0, x1 = _arr(x0, dt), _arr(x1, dt)
    n = x0.size
    z0, z1 = np.empty(n, dt), np.empty(n, dt)
    _fn("orc_sqrt_" + _sfx(x0))(C.c_int64(n), _p(x0), _p(x1), _p(z0), _p(z1))
    return z0, z1


def _eft2(name, a, b):
    dt = np.asarray(a).dtype
    a, b = _arr(a, dt), _arr(b, dt)
    hi, lo = np.empty(a.size, dt), np.empty(a.size, dt)
    _fn("orc_%s_%s" % (name, _sfx(a)))(C.c_int64(a.size), _p(a), _p(b), _p(hi), _p(lo))
    return hi, lo


def two_sum(a, b):
    """Algorithm 1.2: (s, t) with a + b = s + t."""
    return _eft2("two_sum", a, b)


def two_diff(a, b):
    """Algorithm 2.2 (orientation of the lost parts as in Algorithm 2.1)."""
    return _eft2("two_diff", a, b)


def two_prod(a, b):
    """Algorithm 3: (p, e) with a * b = p + e."""
    return _eft2("two_prod", a, b)


def div_rem(a, b):
    """Algorithm 4: (q, r) with a = q b + r."""
    return _eft2("div_rem", a, b)


def sqrt_rem(a):
    """Algorithm 5: (c, d) with a = c^2 + d."""
    dt = np.asarray(a).dtype
    a = _arr(a, dt)
    hi, lo = np.empty(a.size, dt), np.empty(a.size, dt)
    _fn("orc_sqrt_rem_" + _sfx(a))(C.c_int64(a.size), _p(a), _p(hi), _p(lo))
    return hi, lo


def axpy(a, x0, x1, y0, y1):
    """z = MTF1(a, x) then ATF1 with y; ``a`` is the twofold scalar (a0, a1)."""
    dt = np.asarray(x0).dtype
    a = np.ascontiguousarray(np.asarray(a, dtype=dt).reshape(2))
    x0, x1, y0, y1 = (_arr(v, dt) for v in (x0, x1, y0, y1))
    n = x0.size
    z0, z1 = np.empty(n, dt), np.empty(n, dt)
    _fn("orc_axpy_" + _sfx(x0))(C.c_int64(n), _p(a), _p(x0), _p(x1), _p(y0), _p(y1), _p(z0), _p(z1))
    return z0, z1


def horner(c, x0, x1):
    """Horner evaluation of sum c[k] x^k with dotted coefficients c[0..d]."""
    dt = np.asarray(x0).dtype
    c = np.ascontiguousarray(np.asarray(c, dtype=dt))
    x0, x1 = _arr(x0, dt), _arr(x1, dt)
    n = x0.size
    z0, z1 = np.empty(n, dt), np.empty(n, dt)
    _fn("orc_horner_" + _sfx(x0))(C.c_int64(n), C.c_int(c.size - 1), _p(c), _p(x0), _p(x1), _p(z0), _p(z1))
    return z0, z1


def sum(x0, x1=None):  # noqa: A001 - the operation's own name
    """Twofold sum over the fixed pairwise tree; returns (z0, z1) scalars."""
    dt = np.asarray(x0).dtype
    x0, x1 = _arr(x0, dt), _arr(x1, dt)
    out = np.empty(2, dt)
    _fn("orc_sum_" + _sfx(x0))(C.c_int64(x0.size), _p(x0), _p(x1), _p(out))
    return out[0], out[1]


def dot(x0, x1, y0, y1):
    """Twofold dot product over the fixed pairwise tree; returns (z0, z1)."""
    dt = np.asarray(x0).dtype
    x0, x1, y0, y1 = (_arr(v, dt) for v in (x0, x1, y0, y1))
    out = np.empty(2, dt)
    _fn("orc_dot_" + _sfx(x0))(C.c_int64(x0.size), _p(x0), _p(x1), _p(y0), _p(y1), _p(out))
    return out[0], out[1]


def accumulate(steps: int, t0, t1):
    """Sequential ATF1 accumulation of the twofold (t0, t1), ``steps`` times."""
    dt = np.asarray(t0).dtype
    out = np.empty(2, dt)
    ct = C.c_double if dt == np.float64 else C.c_float
    _fn("orc_accumulate_" + _SFX[dt])(C.c_int64(steps), ct(t0), ct(t1), _p(out))
    return out[0], out[1]


# ---- plain counterparts -------------------------------------------------

def plain(op: str, x, y=None):
    """Plain add/sub/mul/div (x, y) or sqrt (x)."""
    dt = np.asarray(x).dtype
    x = _arr(x, dt)
    z = np.empty(x.size, dt)
    if op == "sqrt":
        _fn("orc_plain_sqrt_" + _sfx(x))(C.c_int64(x.size), _p(x), _p(z))
    else:
        y = _arr(y, dt)
        _fn("orc_plain_%s_%s" % (op, _sfx(x)))(C.c_int64(x.size), _p(x), _p(y), _p(z))
    return z


def plain_axpy(a0, x, y):
    dt = np.asarray(x).dtype
    x, y = _arr(x, dt), _arr(y, dt)
    z = np.empty(x.size, dt)
    ct = C.c_double if dt == np.float64 else C.c_float
    _fn("orc_plain_axpy_" + _sfx(x))(C.c_int64(x.size), ct(float(a0)), _p(x), _p(y), _p(z))
    return z


def plain_horner(c, x):
    dt = np.asarray(x).dtype
    c = np.ascontiguousarray(np.asarray(c, dtype=dt))
    x = _arr(x, dt)
    z = np.empty(x.size, dt)
    _fn("orc_plain_horner_" + _sfx(x))(C.c_int64(x.size), C.c_int(c.size - 1), _p(c), _p(x), _p(z))
    return z


def plain_sum(x):
    dt = np.asarray(x).dtype
    x = _arr(x, dt)
    out = np.empty(1, dt)
    _fn("orc_plain_sum_" + _sfx(x))(C.c_int64(x.size), _p(x), _p(out))
    return out[0]


def plain_dot(x, y):
    dt = np.asarray(x).dtype
    x, y = _arr(x, dt), _arr(y, dt)
    out = np.empty(1, dt)
    _fn("orc_plain_dot_" + _sfx(x))(C.c_int64(x.size), _p(x), _p(y), _p(out))
    return out[0]


# ---- FP64 reference deviation for binary32 twofolds ----------------------

def ref64(op: str, *args):
    """Deviation dz0 = z - z0 of binary32 standard results z0, computed from
    the binary64 oracle on the widened inputs.

    ``ref64("add", x0, x1, y0, y1, z0)`` (also sub/mul/div),
    ``ref64("sqrt", x0, x1, z0)``, ``ref64("axpy", a, x0, x1, y0, y1, z0)``,
    ``ref64("horner", c, x0, x1, z0)``, ``ref64("sum", x0, x1, z0)``,
    ``ref64("dot", x0, x1, y0, y1, z0)``.  Returns float64 arrays (a
    one-element array for sum and dot).
    """
    f32 = np.float32
    if op in ("add", "sub", "mul", "div"):
        x0, x1, y0, y1, z0 = (_arr(v, f32) for v in args)
        dz = np.empty(x0.size, np.float64)
        _fn("orc_ref64_" + op)(C.c_int64(x0.size), _p(x0), _p(x1), _p(y0), _p(y1), _p(z0), _p(dz))
    elif op == "sqrt":
        x0, x1, z0 = (_arr(v, f32) for v in args)
        dz = np.empty(x0.size, np.float64)
        _fn("orc_ref64_sqrt")(C.c_int64(x0.size), _p(x0), _p(x1), _p(z0), _p(dz))
    elif op == "axpy":
        a = np.ascontiguousarray(np.asarray(args[0], dtype=f32).reshape(2))
        x0, x1, y0, y1, z0 = (_arr(v, f32) for v in args[1:])
        dz = np.empty(x0.size, np.float64)
        _fn("orc_ref64_axpy")(C.c_int64(x0.size), _p(a), _p(x0), _p(x1), _p(y0), _p(y1), _p(z0), _p(dz))
    elif op == "horner":
        c = np.ascontiguousarray(np.asarray(args[0], dtype=f32))
        x0, x1, z0 = (_arr(v, f32) for v in args[1:])
        dz = np.empty(x0.size, np.float64)
        _fn("orc_ref64_horner")(C.c_int64(x0.size), C.c_int(c.size - 1), _p(c), _p(x0), _p(x1), _p(z0), _p(dz))
    elif op == "sum":
        x0, x1 = _arr(args[0], f32), _arr(args[1], f32)
        z0 = np.asarray([args[2]], f32)
        dz = np.empty(1, np.float64)
        _fn("orc_ref64_sum")(C.c_int64(x0.size), _p(x0), _p(x1), _p(z0), _p(dz))
    elif op == "dot":
        x0, x1, y0, y1 = (_arr(v, f32) for v in args[:4])
        z0 = np.asarray([args[4]], f32)
        dz = np.empty(1, np.float64)
        _fn("orc_ref64_dot")(C.c_int64(x0.size), _p(x0), _p(x1), _p(y0), _p(y1), _p(z0), _p(dz))
    else:
        raise ValueError(op)
    return dz


# ---- coupled algorithms, chains, applications, fma -------------------------

OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4}
MODES = {"twofold": 0, "coupled": 1, "dekker": 2}


def fast_two_sum(a, b):
    """Algorithm 1.1: (s, t), exact when |a| >= |b|."""
    return _eft2("fast_two_sum", a, b)


def coupled(op: str, x0, x1, y0=None, y1=None, renorm: bool = False):
    """Coupled ("p") operation: ATF1 / STF1 for add and sub, MPF1, DPF1,
    RPF1 (and their dotted forms); with ``renorm`` the result is passed
    through Fast Two-Sum (Dekker mode)."""
    dt = np.asarray(x0).dtype
    x0, x1, y0, y1 = (_arr(v, dt) for v in (x0, x1, y0, y1))
    n = x0.size
    z0, z1 = np.empty(n, dt), np.empty(n, dt)
    _fn("orc_coupled_" + _sfx(x0))(C.c_int(OPS[op]), C.c_int(int(renorm)), C.c_int64(n),
                                   _p(x0), _p(x1), _p(y0), _p(y1), _p(z0), _p(z1))
    return z0, z1


def renorm(z0, z1):
    """Fast Two-Sum renormalisation of each twofold."""
    dt = np.asarray(z0).dtype
    z0, z1 = _arr(z0, dt), _arr(z1, dt)
    s, t = np.empty(z0.size, dt), np.empty(z0.size, dt)
    _fn("orc_renorm_" + _sfx(z0))(C.c_int64(z0.size), _p(z0), _p(z1), _p(s), _p(t))
    return s, t


def chain(op: str, mode: str, reps: int, x0, x1, y0=None, y1=None):
    """z = (x0, x1 or +0), then ``reps`` times z = z (op) y (sqrt: sqrt(z))."""
    dt = np.asarray(x0).dtype
    x0, x1, y0, y1 = (_arr(v, dt) for v in (x0, x1, y0, y1))
    n = x0.size
    z0, z1 = np.empty(n, dt), np.empty(n, dt)
    _fn("orc_chain_" + _sfx(x0))(C.c_int(OPS[op]), C.c_int(MODES[mode]), C.c_int64(n), C.c_int64(reps),
                                 _p(x0), _p(x1), _p(y0), _p(y1), _p(z0), _p(z1))
    return z0, z1


def plain_chain(op: str, reps: int, x, y=None):
    dt = np.asarray(x).dtype
    x, y = _arr(x, dt), _arr(y, dt)
    z = np.empty(x.size, dt)
    _fn("orc_plain_chain_" + _sfx(x))(C.c_int(OPS[op]), C.c_int64(x.size), C.c_int64(reps), _p(x), _p(y), _p(z))
    return z


def trsv_upper(m: int, U0, U1, f0, f1):
    """Back-substitution of upper-triangular systems, systems interleaved:
    U[(i*m + j)*nsys + k], f and x [i*nsys + k].  Returns (x0, x1)."""
    dt = np.asarray(U0).dtype
    U0, U1, f0, f1 = (_arr(v, dt) for v in (U0, U1, f0, f1))
    nsys = f0.size // m
    x0, x1 = np.empty(f0.size, dt), np.empty(f0.size, dt)
    _fn("orc_trsv_upper_" + _sfx(U0))(C.c_int64(nsys), C.c_int(m), _p(U0), _p(U1), _p(f0), _p(f1),
                                      _p(x0), _p(x1))
    return x0, x1


def quadratic(a0, a1, b0, b1, c0, c1):
    """Both roots by the school formula; returns (r0, r1, s0, s1) with r the
    root -b - sqrt(.) and s the root -b + sqrt(.) over 2a."""
    dt = np.asarray(a0).dtype
    a0, a1, b0, b1, c0, c1 = (_arr(v, dt) for v in (a0, a1, b0, b1, c0, c1))
    n = a0.size
    out = [np.empty(n, dt) for _ in range(4)]
    _fn("orc_quadratic_" + _sfx(a0))(C.c_int64(n), _p(a0), _p(a1), _p(b0), _p(b1), _p(c0), _p(c1),
                                     *[_p(o) for o in out])
    return tuple(out)


def fma(x0, x1, y0, y1, w0, w1):
    """Twofold fused multiply-add z = x y + w (an extension of the paper)."""
    dt = np.asarray(x0).dtype
    x0, x1, y0, y1, w0, w1 = (_arr(v, dt) for v in (x0, x1, y0, y1, w0, w1))
    n = x0.size
    z0, z1 = np.empty(n, dt), np.empty(n, dt)
    _fn("orc_fma_" + _sfx(x0))(C.c_int64(n), _p(x0), _p(x1), _p(y0), _p(y1), _p(w0), _p(w1), _p(z0), _p(z1))
    return z0, z1


def plain_fma(x, y, w):
    dt = np.asarray(x).dtype
    x, y, w = (_arr(v, dt) for v in (x, y, w))
    z = np.empty(x.size, dt)
    _fn("orc_plain_fma_" + _sfx(x))(C.c_int64(x.size), _p(x), _p(y), _p(w), _p(z))
    return z
