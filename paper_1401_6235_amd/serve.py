"""Python binding of the serving API (tfs_* in include/tf.h).

Argument marshalling only: jobs are plain descriptors handed to the native
server, which admits them, generates their inputs on the GPU and runs
them in the library's persistent kernel.
"""
from __future__ import annotations

import ctypes as C

from . import TF_F32, TF_F64, TF_MAX_DEGREE, TwofoldError, lib

TFS_MAX_SLOTS = 64
TFS_MAX_N = 4096 * 16383  # elements per job: 16383 units of 4096
TFS_OP_SUM, TFS_OP_DOT, TFS_OP_AXPY, TFS_OP_HORNER = 0, 1, 2, 3
TFS_KIND_RANDOM, TFS_KIND_ILLCOND, TFS_KIND_PROVIDED = 0, 1, 2
OPS = {"sum": TFS_OP_SUM, "dot": TFS_OP_DOT, "axpy": TFS_OP_AXPY, "horner": TFS_OP_HORNER}
DTYPES = {"f32": TF_F32, "f64": TF_F64}


class TfsJob(C.Structure):
    _fields_ = [("op", C.c_int), ("dtype", C.c_int), ("kind", C.c_int), ("degree", C.c_int),
                ("n", C.c_int64), ("seed", C.c_uint64), ("a", C.c_double * 2),
                ("c", C.c_double * (TF_MAX_DEGREE + 1)), ("threshold", C.c_double),
                ("x0", C.c_void_p), ("x1", C.c_void_p), ("y0", C.c_void_p), ("y1", C.c_void_p)]


class TfsResult(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int), ("op", C.c_int), ("dtype", C.c_int),
                ("kind", C.c_int), ("flag", C.c_int), ("n", C.c_int64), ("z0", C.c_double),
                ("z1", C.c_double), ("max_abs_z0", C.c_double), ("max_abs_z1", C.c_double),
                ("n_flagged", C.c_uint64), ("nonfinite", C.c_uint64), ("hash_z0", C.c_uint64),
                ("hash_z1", C.c_uint64), ("t_arrive", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_publish", C.c_double), ("t_done", C.c_double), ("queue_us", C.c_double),
                ("gen_us", C.c_double), ("device_us", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TfsStats(C.Structure):
    _fields_ = [("pending", C.c_int64), ("in_flight", C.c_int64), ("completed", C.c_int64),
                ("budget_bytes", C.c_uint64), ("resident_bytes", C.c_uint64),
                ("peak_resident_bytes", C.c_uint64), ("admission_waits", C.c_uint64),
                ("kernel_alive", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _setup():
    L = lib()
    L.tfs_create.restype = C.c_void_p
    L.tfs_create.argtypes = [C.c_int, C.c_uint64, C.c_int]
    L.tfs_submit.restype = C.c_int
    L.tfs_submit.argtypes = [C.c_void_p, C.POINTER(TfsJob), C.c_double, C.POINTER(C.c_uint64)]
    L.tfs_poll.restype = C.c_int
    L.tfs_poll.argtypes = [C.c_void_p, C.POINTER(TfsResult), C.c_int]
    L.tfs_get_stats.restype = C.c_int
    L.tfs_get_stats.argtypes = [C.c_void_p, C.POINTER(TfsStats)]
    L.tfs_clock.restype = C.c_double
    L.tfs_destroy.restype = C.c_int
    L.tfs_destroy.argtypes = [C.c_void_p]
    return L


def tfs_clock() -> float:
    return float(_setup().tfs_clock())


def make_job(op, dtype, n, seed=0, kind=TFS_KIND_RANDOM, a=(0.7, 1e-17), c=None, threshold=0.0,
             x0=None, x1=None, y0=None, y1=None) -> TfsJob:
    """A job descriptor.  op: 'sum' | 'dot' | 'axpy' | 'horner' (or code);
    dtype: 'f32' | 'f64' (or code); inputs x0.. are device tensors for
    TFS_KIND_PROVIDED jobs."""
    j = TfsJob()
    j.op = OPS.get(op, op)
    j.dtype = DTYPES.get(dtype, dtype)
    j.kind = kind
    j.n = int(n)
    j.seed = int(seed) & (2 ** 64 - 1)
    j.a[0], j.a[1] = float(a[0]), float(a[1])
    coef = list(c) if c is not None else []
    j.degree = max(0, len(coef) - 1)
    for k, v in enumerate(coef):
        j.c[k] = float(v)
    j.threshold = float(threshold)
    for name, t in (("x0", x0), ("x1", x1), ("y0", y0), ("y1", y1)):
        setattr(j, name, None if t is None else t.data_ptr())
    return j


class Server:
    """A serving instance (tfs_create .. tfs_destroy)."""

    def __init__(self, device: int = 0, budget_bytes: int = 64 << 30, max_slots: int = TFS_MAX_SLOTS):
        self._L = _setup()
        self._h = self._L.tfs_create(device, budget_bytes, max_slots)
        if not self._h:
            raise TwofoldError("tfs_create failed (device %d, budget %d)" % (device, budget_bytes))
        self._keep = {}

    def submit(self, job: TfsJob, t_arrive: float = 0.0, keep=None) -> int:
        """Queue a job; `keep` holds objects (input tensors) alive until the
        job's result has been polled."""
        jid = C.c_uint64(0)
        st = self._L.tfs_submit(self._h, C.byref(job), C.c_double(t_arrive), C.byref(jid))
        if st != 0:
            raise TwofoldError("tfs_submit failed: %s (%d)" % (lib().tf_strerror(st).decode(), st))
        if keep is not None:
            self._keep[jid.value] = keep
        return jid.value

    def poll(self, max_results: int = 256):
        buf = (TfsResult * max_results)()
        k = self._L.tfs_poll(self._h, buf, max_results)
        out = [buf[i].as_dict() for i in range(k)]
        for r in out:
            self._keep.pop(r["id"], None)
        return out

    def stats(self):
        s = TfsStats()
        self._L.tfs_get_stats(self._h, C.byref(s))
        return s.as_dict()

    def close(self):
        if self._h:
            self._L.tfs_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_stream(srv: "Server", times, jobs, keep=None, t0_delay: float = 0.05, timeout: float = 120.0):
    """Submit jobs[k] at tfs_clock() time t0 + times[k] (busy-waiting on the
    clock, polling completions in between) and wait for all results.
    Returns (ids, {id: result}); arrival times are the scheduled ones, so
    any lateness of this submitting loop counts against the measured latency."""
    import time as _time
    t0 = tfs_clock() + t0_delay
    ids, results = [], {}
    for k, (t, job) in enumerate(zip(times, jobs)):
        ta = t0 + t
        while tfs_clock() < ta:
            pass
        ids.append(srv.submit(job, t_arrive=ta, keep=None if keep is None else keep[k]))
        for r in srv.poll():
            results[r["id"]] = r
    deadline = _time.time() + timeout
    while len(results) < len(ids) and _time.time() < deadline:
        for r in srv.poll():
            results[r["id"]] = r
        _time.sleep(0.001)
    return ids, results
