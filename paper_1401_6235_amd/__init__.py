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


def _out(z, like):
    return _torch().empty_like(like) if z is None else z


# ---------------------------------------------------------------------------
# elementwise
# ---------------------------------------------------------------------------

def _binary(name, x0, x1, y0, y1, z0, z1, stream):
    n = x0.numel()
    code = _dtype_code(x0)
    z0, z1 = _out(z0, x0), _out(z1, x0)
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
    z0, z1 = _out(z0, x0), _out(z1, x0)
    st = lib().tf_sqrt(C.c_int(_dtype_code(x0)), C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype),
                       _ptr(z0, n, x0.dtype), _ptr(z1, n, x0.dtype), _stream(stream))
    _check(st, "tf_sqrt")
    return z0, z1


def tf_axpy(a, x0, x1, y0, y1, z0=None, z1=None, stream=None):
    """z = a x + y with a twofold scalar a = (a0, a1)."""
    n = x0.numel()
    code = _dtype_code(x0)
    ha, pa = _host_array(a, code)
    z0, z1 = _out(z0, x0), _out(z1, x0)
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
    z0, z1 = _out(z0, x0), _out(z1, x0)
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


def workspace(x0, n=None):
    """A workspace tensor large enough for a reduction over x0."""
    torch = _torch()
    n = x0.numel() if n is None else n
    b = tf_reduce_workspace_bytes(_dtype_code(x0), n)
    return torch.empty(max(b, 1), dtype=torch.uint8, device=x0.device)


def tf_sum(x0, x1=None, out=None, work=None, stream=None):
    """Twofold sum; returns a 2-element device tensor (z0, z1)."""
    n = x0.numel()
    out = _torch().empty(2, dtype=x0.dtype, device=x0.device) if out is None else out
    work = workspace(x0) if work is None else work
    st = lib().tf_sum(C.c_int(_dtype_code(x0)), C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype),
                      _ptr(out, 2, x0.dtype), _ptr(work), C.c_size_t(work.numel() * work.element_size()),
                      _stream(stream))
    _check(st, "tf_sum")
    return out


def tf_dot(x0, x1, y0, y1, out=None, work=None, stream=None):
    """Twofold dot product; returns a 2-element device tensor (z0, z1)."""
    n = x0.numel()
    out = _torch().empty(2, dtype=x0.dtype, device=x0.device) if out is None else out
    work = workspace(x0) if work is None else work
    st = lib().tf_dot(C.c_int(_dtype_code(x0)), C.c_int64(n), _ptr(x0, n), _ptr(x1, n, x0.dtype),
                      _ptr(y0, n, x0.dtype), _ptr(y1, n, x0.dtype), _ptr(out, 2, x0.dtype), _ptr(work),
                      C.c_size_t(work.numel() * work.element_size()), _stream(stream))
    _check(st, "tf_dot")
    return out


# ---------------------------------------------------------------------------
# plain counterparts and the memory probe
# ---------------------------------------------------------------------------

def _plain2(name, x, y, z, stream):
    n = x.numel()
    z = _out(z, x)
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
    z = _out(z, x)
    st = lib().tf_plain_sqrt(C.c_int(_dtype_code(x)), C.c_int64(n), _ptr(x, n), _ptr(z, n, x.dtype),
                             _stream(stream))
    _check(st, "tf_plain_sqrt")
    return z


def tf_plain_axpy(a0, x, y, z=None, stream=None):
    n = x.numel()
    code = _dtype_code(x)
    ha, pa = _host_array([a0], code)
    z = _out(z, x)
    st = lib().tf_plain_axpy(C.c_int(code), C.c_int64(n), pa, _ptr(x, n), _ptr(y, n, x.dtype),
                             _ptr(z, n, x.dtype), _stream(stream))
    _check(st, "tf_plain_axpy")
    return z


def tf_plain_horner(c, x, z=None, stream=None):
    n = x.numel()
    code = _dtype_code(x)
    hc, pc = _host_array(c, code)
    z = _out(z, x)
    st = lib().tf_plain_horner(C.c_int(code), C.c_int64(n), C.c_int(hc.numel() - 1), pc, _ptr(x, n),
                               _ptr(z, n, x.dtype), _stream(stream))
    _check(st, "tf_plain_horner")
    return z


def tf_plain_sum(x, out=None, work=None, stream=None):
    n = x.numel()
    out = _torch().empty(1, dtype=x.dtype, device=x.device) if out is None else out
    work = workspace(x) if work is None else work
    st = lib().tf_plain_sum(C.c_int(_dtype_code(x)), C.c_int64(n), _ptr(x, n), _ptr(out, 1, x.dtype),
                            _ptr(work), C.c_size_t(work.numel() * work.element_size()), _stream(stream))
    _check(st, "tf_plain_sum")
    return out


def tf_plain_dot(x, y, out=None, work=None, stream=None):
    n = x.numel()
    out = _torch().empty(1, dtype=x.dtype, device=x.device) if out is None else out
    work = workspace(x) if work is None else work
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
