"""Twofold fast arithmetic on AMD Instinct MI355X: Python binding.

Thin ctypes binding of ``libtwofold.so`` (the C ABI declared in
``include/tf.h``): every function has the C name, takes torch tensors that
live on the GPU, passes their device pointers and the current HIP stream,
and raises on a non-zero status.  Only argument marshalling happens here;
every step of the computation runs in the library's HIP kernels.  torch is
used for device memory and streams only.

The library must have been built (``paper_1401_6235_amd.build.build()``);
nothing here falls back to any other implementation.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtwofold.so")

TF_F32 = 1
TF_F64 = 2
TF_OK = 0
TF_MAX_DEGREE = 32
TF_CFG_EW_BLOCKS_PER_CU = 1
TF_CFG_RED_TILES_PER_BLOCK = 2
TF_CFG_RED_WAVES = 3
TF_MAX_TRSV = 64
TF_NOALLOC_SCRATCH_BYTES = 4 << 20
TF_OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4}
TF_MODES = {"twofold": 0, "coupled": 1, "dekker": 2}

_lib = None


class TwofoldError(RuntimeError):
    pass


def lib() -> C.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TwofoldError(
                "libtwofold.so is missing: build it with paper_1401_6235_amd.build.build() "
                "(hipcc, gfx950) before using the library")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded (one runtime per process), not to a second copy from the
        # system path that would not know torch's device memory
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        _lib = C.CDLL(LIB_PATH)
        _lib.tf_strerror.restype = C.c_char_p
        _lib.tf_reduce_workspace_bytes.restype = C.c_size_t
        _lib.tf_reduce_workspace_bytes.argtypes = [C.c_int, C.c_int64]
        _lib.tf_config.restype = C.c_int64
        _lib.tf_config.argtypes = [C.c_int, C.c_int64]
    return _lib


def _check(status: int, what: str):
    if status != TF_OK:
        raise TwofoldError("%s failed: %s (%d)" % (what, lib().tf_strerror(status).decode(), status))


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return TF_F64
    if t.dtype == torch.float32:
        return TF_F32
    raise TypeError("twofold arrays are float64 or float32, got %s" % t.dtype)


def _ptr(t, n=None, dtype=None):
    """Device pointer of a contiguous GPU tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError("length mismatch: %d != %d" % (t.numel(), n))
    if dtype is not None and t.dtype != dtype:
        raise TypeError("dtype mismatch: %s != %s" % (t.dtype, dtype))
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _host_array(values, code):
    torch = _torch()
    dt = torch.float64 if code == TF_F64 else torch.float32
    t = torch.as_tensor(values, dtype=dt).contiguous().cpu()
    return t, C.c_void_p(t.data_ptr())


def _on(stream):
    """Context for buffers made here: allocated on the stream whose kernels
    use them, so torch's caching allocator cannot hand their memory to other
    work while those kernels may still read or write it."""
    return contextlib.nullcontext() if stream is None else _torch().cuda.stream(stream)


def _out(z, like, stream=None):
    if z is not None:
        return z
    with _on(stream):
        return _torch().empty_like(like)


def _empty(count, like, stream=None):
    with _on(stream):
        return _torch().empty(count, dtype=like.dtype, device=like.device)


# ---------------------------------------------------------------------------
# elementwise
# ---------------------------------------------------------------------------

def _binary(name, x0, x1, y0, y1, z0, z1, stream):
    n = x0.numel()
    code = _dtype_code(x0)
    z0, z1 = _out(z0, x0, stream), _out(z1, x0, stream)
    st = getattr(lib(), name)(C.c_int(code), C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype),
                              _ptr(y0, n, x0.dtype), _ptr(y1, n, x0.dtype), _ptr(z0, n, x0.dtype),
                              _ptr(z1, n, x0.dtype), _stream(stream))
    _check(st, name)
    return z0, z1


def tf_add(x0, x1, y0, y1, z0=None, z1=None, stream=None):
    """Twofold add (ATF1 family); x1 / y1 None = dotted operand."""
    return _binary("tf_add", x0, x1, y0, y1, z0, z1, stream)


def tf_sub(x0, x1, y0, y1, z0=None, z1=None, stream=None):
    """Twofold subtract (STF1 family)."""
    return _binary("tf_sub", x0, x1, y0, y1, z0, z1, stream)


def tf_mul(x0, x1, y0, y1, z0=None, z1=None, stream=None):
    """Twofold multiply (MTF1 family)."""
    return _binary("tf_mul", x0, x1, y0, y1, z0, z1, stream)


def tf_div(x0, x1, y0, y1, z0=None, z1=None, stream=None):
    """Twofold divide (DTF1 family)."""
    return _binary("tf_div", x0, x1, y0, y1, z0, z1, stream)


def tf_sqrt(x0, x1, z0=None, z1=None, stream=None):
    """Twofold square root (RTF1 / RPF1.1)."""
    n = x0.numel()
    z0, z1 = _out(z0, x0, stream), _out(z1, x0, stream)
    st = lib().tf_sqrt(C.c_int(_dtype_code(x0)), C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype),
                       _ptr(z0, n, x0.dtype), _ptr(z1, n, x0.dtype), _stream(stream))
    _check(st, "tf_sqrt")
    return z0, z1


def tf_axpy(a, x0, x1, y0, y1, z0=None, z1=None, stream=None):
    """z = a x + y with a twofold scalar a = (a0, a1)."""
    n = x0.numel()
    code = _dtype_code(x0)
    ha, pa = _host_array(a, code)
    z0, z1 = _out(z0, x0, stream), _out(z1, x0, stream)
    st = lib().tf_axpy(C.c_int(code), C.c_int64(n), pa, _ptr(x0, n), _ptr(x1, n, x0.dtype),
                       _ptr(y0, n, x0.dtype), _ptr(y1, n, x0.dtype), _ptr(z0, n, x0.dtype),
                       _ptr(z1, n, x0.dtype), _stream(stream))
    _check(st, "tf_axpy")
    return z0, z1


def tf_horner(c, x0, x1, z0=None, z1=None, stream=None):
    """Horner evaluation of sum c[k] x^k (c dotted, length degree + 1)."""
    n = x0.numel()
    code = _dtype_code(x0)
    hc, pc = _host_array(c, code)
    z0, z1 = _out(z0, x0, stream), _out(z1, x0, stream)
    st = lib().tf_horner(C.c_int(code), C.c_int64(n), C.c_int(hc.numel() - 1), pc, _ptr(x0, n),
                         _ptr(x1, n, x0.dtype), _ptr(z0, n, x0.dtype), _ptr(z1, n, x0.dtype),
                         _stream(stream))
    _check(st, "tf_horner")
    return z0, z1


# ---------------------------------------------------------------------------
# reductions
# ---------------------------------------------------------------------------

def tf_reduce_workspace_bytes(dtype_code: int, n: int) -> int:
    return int(lib().tf_reduce_workspace_bytes(dtype_code, n))


def workspace(x0, n=None, stream=None):
    """A workspace tensor large enough for a reduction over x0, allocated on
    ``stream`` (default: the current stream), the stream the reduction that
    uses it must run on."""
    torch = _torch()
    n = x0.numel() if n is None else n
    b = tf_reduce_workspace_bytes(_dtype_code(x0), n)
    with _on(stream):
        return torch.empty(max(b, 1), dtype=torch.uint8, device=x0.device)


def tf_sum(x0, x1=None, out=None, work=None, stream=None):
    """Twofold sum; returns a 2-element device tensor (z0, z1)."""
    n = x0.numel()
    out = _empty(2, x0, stream) if out is None else out
    work = workspace(x0, stream=stream) if work is None else work
    st = lib().tf_sum(C.c_int(_dtype_code(x0)), C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype),
                      _ptr(out, 2, x0.dtype), _ptr(work), C.c_size_t(work.numel() * work.element_size()),
                      _stream(stream))
    _check(st, "tf_sum")
    return out


def tf_dot(x0, x1, y0, y1, out=None, work=None, stream=None):
    """Twofold dot product; returns a 2-element device tensor (z0, z1)."""
    n = x0.numel()
    out = _empty(2, x0, stream) if out is None else out
    work = workspace(x0, stream=stream) if work is None else work
    st = lib().tf_dot(C.c_int(_dtype_code(x0)), C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype),
                      _ptr(y0, n, x0.dtype), _ptr(y1, n, x0.dtype), _ptr(out, 2, x0.dtype), _ptr(work),
                      C.c_size_t(work.numel() * work.element_size()), _stream(stream))
    _check(st, "tf_dot")
    return out


def tf_dot_noalloc(x0, x1, y0, y1, out, stream=None):
    """tf_dot with the partials in the library's static device array: no
    workspace, no allocation (``out``, 2 elements of x0's dtype on the
    device, is required).  Calls that overlap on one GPU race."""
    n = x0.numel()
    st = lib().tf_dot_noalloc(C.c_int(_dtype_code(x0)), C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype),
                              _ptr(y0, n, x0.dtype), _ptr(y1, n, x0.dtype), _ptr(out, 2, x0.dtype),
                              _stream(stream))
    _check(st, "tf_dot_noalloc")
    return out


# ---------------------------------------------------------------------------
# plain counterparts and the memory probe
# ---------------------------------------------------------------------------

def _plain2(name, x, y, z, stream):
    n = x.numel()
    z = _out(z, x, stream)
    st = getattr(lib(), name)(C.c_int(_dtype_code(x)), C.c_int64(n), _ptr(x, n), _ptr(y, n, x.dtype),
                              _ptr(z, n, x.dtype), _stream(stream))
    _check(st, name)
    return z


def tf_plain_add(x, y, z=None, stream=None):
    return _plain2("tf_plain_add", x, y, z, stream)


def tf_plain_sub(x, y, z=None, stream=None):
    return _plain2("tf_plain_sub", x, y, z, stream)


def tf_plain_mul(x, y, z=None, stream=None):
    return _plain2("tf_plain_mul", x, y, z, stream)


def tf_plain_div(x, y, z=None, stream=None):
    return _plain2("tf_plain_div", x, y, z, stream)


def tf_vmem(x, y, z=None, stream=None):
    return _plain2("tf_vmem", x, y, z, stream)


def tf_plain_sqrt(x, z=None, stream=None):
    n = x.numel()
    z = _out(z, x, stream)
    st = lib().tf_plain_sqrt(C.c_int(_dtype_code(x)), C.c_int64(n), _ptr(x, n), _ptr(z, n, x.dtype),
                             _stream(stream))
    _check(st, "tf_plain_sqrt")
    return z


def tf_plain_axpy(a0, x, y, z=None, stream=None):
    n = x.numel()
    code = _dtype_code(x)
    ha, pa = _host_array([a0], code)
    z = _out(z, x, stream)
    st = lib().tf_plain_axpy(C.c_int(code), C.c_int64(n), pa, _ptr(x, n), _ptr(y, n, x.dtype),
                             _ptr(z, n, x.dtype), _stream(stream))
    _check(st, "tf_plain_axpy")
    return z


def tf_plain_horner(c, x, z=None, stream=None):
    n = x.numel()
    code = _dtype_code(x)
    hc, pc = _host_array(c, code)
    z = _out(z, x, stream)
    st = lib().tf_plain_horner(C.c_int(code), C.c_int64(n), C.c_int(hc.numel() - 1), pc, _ptr(x, n),
                               _ptr(z, n, x.dtype), _stream(stream))
    _check(st, "tf_plain_horner")
    return z


def tf_plain_sum(x, out=None, work=None, stream=None):
    n = x.numel()
    out = _empty(1, x, stream) if out is None else out
    work = workspace(x, stream=stream) if work is None else work
    st = lib().tf_plain_sum(C.c_int(_dtype_code(x)), C.c_int64(n), _ptr(x, n), _ptr(out, 1, x.dtype),
                            _ptr(work), C.c_size_t(work.numel() * work.element_size()), _stream(stream))
    _check(st, "tf_plain_sum")
    return out


def tf_plain_dot(x, y, out=None, work=None, stream=None):
    n = x.numel()
    out = _empty(1, x, stream) if out is None else out
    work = workspace(x, stream=stream) if work is None else work
    st = lib().tf_plain_dot(C.c_int(_dtype_code(x)), C.c_int64(n), _ptr(x, n), _ptr(y, n, x.dtype),
                            _ptr(out, 1, x.dtype), _ptr(work), C.c_size_t(work.numel() * work.element_size()),
                            _stream(stream))
    _check(st, "tf_plain_dot")
    return out


def tf_config(key: int, value: int) -> int:
    """Set a launch-tuning knob (results never depend on it); returns the
    previous value."""
    old = int(lib().tf_config(key, value))
    if old < 0:
        raise TwofoldError("tf_config(%d, %d): invalid key or value" % (key, value))
    return old


# ---------------------------------------------------------------------------
# coupled algorithms, renormalisation, chains
# ---------------------------------------------------------------------------

def tf_coupled(op, x0, x1, y0=None, y1=None, renorm=False, z0=None, z1=None, stream=None):
    """Coupled operation (ATF1, STF1, MPF1, DPF1, RPF1); ``renorm`` adds Fast
    Two-Sum (Dekker mode).  ``op`` is "add", "sub", "mul", "div" or "sqrt"."""
    n = x0.numel()
    z0, z1 = _out(z0, x0, stream), _out(z1, x0, stream)
    st = lib().tf_coupled(C.c_int(_dtype_code(x0)), C.c_int(TF_OPS[op]), C.c_int(int(bool(renorm))),
                          C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype), _ptr(y0, n, x0.dtype),
                          _ptr(y1, n, x0.dtype), _ptr(z0, n, x0.dtype), _ptr(z1, n, x0.dtype), _stream(stream))
    _check(st, "tf_coupled")
    return z0, z1


def tf_renorm(z0, z1, s=None, t=None, stream=None):
    """Fast Two-Sum renormalisation of each twofold."""
    n = z0.numel()
    s, t = _out(s, z0, stream), _out(t, z0, stream)
    st = lib().tf_renorm(C.c_int(_dtype_code(z0)), C.c_int64(n), _ptr(z0, n), _ptr(z1, n, z0.dtype),
                         _ptr(s, n, z0.dtype), _ptr(t, n, z0.dtype), _stream(stream))
    _check(st, "tf_renorm")
    return s, t


def tf_chain(op, mode, reps, x0, x1, y0=None, y1=None, z0=None, z1=None, stream=None):
    """z = (x0, x1 or +0), then ``reps`` times z = z op y (sqrt: sqrt(z)),
    in registers; ``mode`` is "twofold", "coupled" or "dekker"."""
    n = x0.numel()
    z0, z1 = _out(z0, x0, stream), _out(z1, x0, stream)
    st = lib().tf_chain(C.c_int(_dtype_code(x0)), C.c_int(TF_OPS[op]), C.c_int(TF_MODES[mode]), C.c_int64(n),
                        C.c_int64(reps), _ptr(x0, n), _ptr(x1, n, x0.dtype), _ptr(y0, n, x0.dtype),
                        _ptr(y1, n, x0.dtype), _ptr(z0, n, x0.dtype), _ptr(z1, n, x0.dtype), _stream(stream))
    _check(st, "tf_chain")
    return z0, z1


def tf_plain_chain(op, reps, x, y=None, z=None, stream=None):
    n = x.numel()
    z = _out(z, x, stream)
    st = lib().tf_plain_chain(C.c_int(_dtype_code(x)), C.c_int(TF_OPS[op]), C.c_int64(n), C.c_int64(reps),
                              _ptr(x, n), _ptr(y, n, x.dtype), _ptr(z, n, x.dtype), _stream(stream))
    _check(st, "tf_plain_chain")
    return z


# ---------------------------------------------------------------------------
# applications
# ---------------------------------------------------------------------------

def tf_trsv_upper(m, U0, U1, f0, f1=None, x0=None, x1=None, stream=None):
    """Back-substitution of upper-triangular m x m systems, interleaved:
    U[(i*m + j)*nsys + k], f and x [i*nsys + k]."""
    nsys = f0.numel() // m
    x0, x1 = _out(x0, f0, stream), _out(x1, f0, stream)
    st = lib().tf_trsv_upper(C.c_int(_dtype_code(f0)), C.c_int64(nsys), C.c_int(m),
                             _ptr(U0, m * m * nsys, f0.dtype), _ptr(U1, m * m * nsys, f0.dtype),
                             _ptr(f0, m * nsys), _ptr(f1, m * nsys, f0.dtype), _ptr(x0, m * nsys, f0.dtype),
                             _ptr(x1, m * nsys, f0.dtype), _stream(stream))
    _check(st, "tf_trsv_upper")
    return x0, x1


def tf_plain_trsv_upper(m, U, f, x=None, stream=None):
    nsys = f.numel() // m
    x = _out(x, f, stream)
    st = lib().tf_plain_trsv_upper(C.c_int(_dtype_code(f)), C.c_int64(nsys), C.c_int(m),
                                   _ptr(U, m * m * nsys, f.dtype), _ptr(f, m * nsys), _ptr(x, m * nsys, f.dtype),
                                   _stream(stream))
    _check(st, "tf_plain_trsv_upper")
    return x


def tf_quadratic(a0, a1, b0, b1, c0, c1, out=None, stream=None):
    """Both roots (r0, r1, s0, s1) of a x^2 + b x + c = 0, twofold operands."""
    n = a0.numel()
    out = tuple(_out(None, a0, stream) for _ in range(4)) if out is None else out
    st = lib().tf_quadratic(C.c_int(_dtype_code(a0)), C.c_int64(n),
                            *[_ptr(v, n, a0.dtype) for v in (a0, a1, b0, b1, c0, c1)],
                            *[_ptr(v, n, a0.dtype) for v in out], _stream(stream))
    _check(st, "tf_quadratic")
    return out


def tf_plain_quadratic(a, b, c, r=None, s=None, stream=None):
    n = a.numel()
    r, s = _out(r, a, stream), _out(s, a, stream)
    st = lib().tf_plain_quadratic(C.c_int(_dtype_code(a)), C.c_int64(n),
                                  *[_ptr(v, n, a.dtype) for v in (a, b, c, r, s)], _stream(stream))
    _check(st, "tf_plain_quadratic")
    return r, s


def tf_fma(x0, x1, y0, y1, w0, w1, z0=None, z1=None, stream=None):
    """Twofold fused multiply-add z = x y + w; None low parts are dotted."""
    n = x0.numel()
    z0, z1 = _out(z0, x0, stream), _out(z1, x0, stream)
    st = lib().tf_fma(C.c_int(_dtype_code(x0)), C.c_int64(n),
                      *[_ptr(v, n, x0.dtype) for v in (x0, x1, y0, y1, w0, w1, z0, z1)], _stream(stream))
    _check(st, "tf_fma")
    return z0, z1


def tf_plain_fma(x, y, w, z=None, stream=None):
    n = x.numel()
    z = _out(z, x, stream)
    st = lib().tf_plain_fma(C.c_int(_dtype_code(x)), C.c_int64(n),
                            *[_ptr(v, n, x.dtype) for v in (x, y, w, z)], _stream(stream))
    _check(st, "tf_plain_fma")
    return z
