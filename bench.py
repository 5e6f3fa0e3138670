#!/usr/bin/env python3
"""Benchmark of the twofold hot path on one MI355X.

One step = one pass of every twofold kernel of the hot path over resident
synthetic inputs, binary64 and binary32:
    add, sub, mul, div, sqrt   (both operands twofold)   n = 2^28
    axpy  (a = (0.7, 1e-17))                             n = 2^28
    Horner, degree 8                                     n = 2^28
    sum (twofold leaves), dot (plain vectors)            n = 2^26, cond 1e16
The same pass with the plain (non-twofold) kernels and the memory probe is
timed right after, for the twofold/plain slowdown.  Then, outside the step:
the dotted and mixed operand forms at n = 2^28 (one operand dotted, both
dotted: the exact transforms, the dotted square root) against the same plain
kernels; the in-register chains (every operation, twofold / coupled / Dekker, against
the plain chain: the paper's in-cache criterion), the batched applications
and the fma, each against its plain kernel, and the paper's own slowdowns
as context; then the serving stream (20,000 verification jobs at 2,000
jobs/s on the persistent kernel) with p50 / p99 latency, throughput and
flag counts.  value = twofold elements per second over the step (input
elements for the reductions).

Per-kernel durations come from HIP events on the launch stream around each
kernel, averaged over the timed steps.  The roofline entry is for the
kernel with the longest average duration, with algorithmic bytes per
element stated in KERNELS below; "traffic" is read from the committed
rocprofv3 counter summary when that summary was taken on the current kernel
source, else null.  cpu_baseline times the scalar oracle on a bounded
sample of the same workload on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
N_STREAM = 1 << 28
N_REDUCE = 1 << 26
REDUCE_COND = 1e16
HORNER_DEGREE = 8

# name -> (algorithmic bytes per element in units of the element size,
#          plain counterpart)
KERNELS = {
    "add": (6, "plain_add"),
    "sub": (6, "plain_sub"),
    "mul": (6, "plain_mul"),
    "div": (6, "plain_div"),
    "sqrt": (4, "plain_sqrt"),
    "axpy": (6, "plain_axpy"),
    "horner": (4, "plain_horner"),
    "sum": (2, "plain_sum"),
    "dot": (2, "plain_dot"),
}
PLAIN_WORDS = {"plain_add": 3, "plain_sub": 3, "plain_mul": 3, "plain_div": 3, "plain_sqrt": 2,
               "plain_axpy": 3, "plain_horner": 2, "plain_sum": 1, "plain_dot": 2, "vmem": 3}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def strip_comments(src: str) -> str:
    """C++ source without its comments (string and character literals kept
    as they are), each comment replaced by one space."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return "".join(out)


def kernel_source_hash() -> str:
    """Hash of the code the profiled kernels are built from: every HIP
    source and header of the library except the serving loop's
    (tf_serve*), which none of the step, chain or application kernels
    includes, with comments left out (a comment edit does not change the
    kernels, so it keeps the profiles valid)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1401_6235_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")) and not name.startswith("tf_serve"):
            h.update(strip_comments(open(os.path.join(csrc, name)).read()).encode())
    return h.hexdigest()[:16]


def make_inputs(torch, dtype_np, W):
    """Resident device inputs for one working type."""
    import numpy as np
    dev = "cuda"

    def g(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    log("generating %s inputs (n=2^28 elementwise, 2^26 reductions)" % np.dtype(dtype_np))
    c = W.elementwise("add", N_STREAM, seed=0, dtype=dtype_np)
    d = {k: g(v) for k, v in c.items()}
    del c
    s = W.elementwise("sqrt", N_STREAM, seed=0, dtype=dtype_np)
    d["s0"], d["s1"] = g(s["x0"]), g(s["x1"])
    del s
    h = W.horner_case(N_STREAM, seed=0, dtype=dtype_np, degree=HORNER_DEGREE)
    d["h0"], d["h1"], d["c"] = g(h["x0"]), g(h["x1"]), h["c"]
    del h
    r = W.illdot_case(N_REDUCE, REDUCE_COND, seed=0, dtype=dtype_np)
    hi, lo = W.product_split(r["x"], r["y"])
    d["rx"], d["ry"], d["rhi"], d["rlo"] = g(r["x"]), g(r["y"]), g(hi), g(lo)
    d["cond"] = r["cond"]
    del r, hi, lo
    d["a"] = W.axpy_case(1, dtype=dtype_np)["a"]
    d["z0"] = torch.empty_like(d["x0"])
    d["z1"] = torch.empty_like(d["x0"])
    d["out"] = torch.empty(2, dtype=d["x0"].dtype, device=dev)
    import paper_1401_6235_amd as tf
    d["work"] = tf.workspace(d["rx"])
    return d


def twofold_calls(tf, d):
    z0, z1 = d["z0"], d["z1"]
    return [
        ("add", N_STREAM, lambda: tf.tf_add(d["x0"], d["x1"], d["y0"], d["y1"], z0, z1)),
        ("sub", N_STREAM, lambda: tf.tf_sub(d["x0"], d["x1"], d["y0"], d["y1"], z0, z1)),
        ("mul", N_STREAM, lambda: tf.tf_mul(d["x0"], d["x1"], d["y0"], d["y1"], z0, z1)),
        ("div", N_STREAM, lambda: tf.tf_div(d["x0"], d["x1"], d["y0"], d["y1"], z0, z1)),
        ("sqrt", N_STREAM, lambda: tf.tf_sqrt(d["s0"], d["s1"], z0, z1)),
        ("axpy", N_STREAM, lambda: tf.tf_axpy(d["a"], d["x0"], d["x1"], d["y0"], d["y1"], z0, z1)),
        ("horner", N_STREAM, lambda: tf.tf_horner(d["c"], d["h0"], d["h1"], z0, z1)),
        ("sum", N_REDUCE, lambda: tf.tf_sum(d["rhi"], d["rlo"], d["out"], d["work"])),
        ("dot", N_REDUCE, lambda: tf.tf_dot(d["rx"], None, d["ry"], None, d["out"], d["work"])),
    ]


def plain_calls(tf, d):
    z = d["z0"]
    return [
        ("plain_add", N_STREAM, lambda: tf.tf_plain_add(d["x0"], d["y0"], z)),
        ("plain_sub", N_STREAM, lambda: tf.tf_plain_sub(d["x0"], d["y0"], z)),
        ("plain_mul", N_STREAM, lambda: tf.tf_plain_mul(d["x0"], d["y0"], z)),
        ("plain_div", N_STREAM, lambda: tf.tf_plain_div(d["x0"], d["y0"], z)),
        ("plain_sqrt", N_STREAM, lambda: tf.tf_plain_sqrt(d["s0"], z)),
        ("plain_axpy", N_STREAM, lambda: tf.tf_plain_axpy(float(d["a"][0]), d["x0"], d["y0"], z)),
        ("plain_horner", N_STREAM, lambda: tf.tf_plain_horner(d["c"], d["h0"], z)),
        ("plain_sum", N_REDUCE, lambda: tf.tf_plain_sum(d["rhi"], d["out"][:1], d["work"])),
        ("plain_dot", N_REDUCE, lambda: tf.tf_plain_dot(d["rx"], d["ry"], d["out"][:1], d["work"])),
        ("vmem", N_STREAM, lambda: tf.tf_vmem(d["x0"], d["y0"], z)),
    ]


def run_pass(torch, calls, steps, warmup):
    """Warm up, then time `steps` passes: wall time of the whole pass
    (synchronised on both sides) and HIP-event time of every call."""
    for _ in range(warmup):
        for _, _, fn in calls:
            fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in calls] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        for k, (_, _, fn) in enumerate(calls):
            ev[s][k][0].record(stream)
            fn()
            ev[s][k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = {}
    for k, (name, n, _) in enumerate(calls):
        ms = [ev[s][k][0].elapsed_time(ev[s][k][1]) for s in range(steps)]
        per[name] = {"n": n, "ms_avg": sum(ms) / len(ms), "ms_min": min(ms)}
    return wall, per


def traffic_for(kernel_key: str, src_hash: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("source_hash") != src_hash:
        return None
    k = t.get("kernels", {}).get(kernel_key)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(W, seconds_target=15.0):
    """The oracle (scalar C, loaded with ctypes) on a bounded sample of the
    step: every kernel of the step on n = 2^20 elements (2^20 leaves for
    the reductions), binary64 and binary32, timed on one thread and then on
    every host core.  The all-core run partitions each call into one
    contiguous chunk per thread (independent elements; for sum and dot,
    subtrees of the tree when the thread count is a power of two, the final
    join of the per-thread results left out); ctypes releases the
    interpreter lock, so the chunks run in parallel.  value is the all-core
    rate."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import oracle
    n = 1 << 20
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    jobs_by_type = []
    for dt in (np.float64, np.float32):
        c = W.elementwise("add", n, seed=0, dtype=dt)
        s = W.elementwise("sqrt", n, seed=0, dtype=dt)
        h = W.horner_case(n, seed=0, dtype=dt)
        r = W.illdot_case(n, REDUCE_COND, seed=0, dtype=dt)
        hi, lo = W.product_split(r["x"], r["y"])
        a = W.axpy_case(1, dtype=dt)["a"]
        jobs_by_type.append([
            lambda i, j, c=c: oracle.add(c["x0"][i:j], c["x1"][i:j], c["y0"][i:j], c["y1"][i:j]),
            lambda i, j, c=c: oracle.sub(c["x0"][i:j], c["x1"][i:j], c["y0"][i:j], c["y1"][i:j]),
            lambda i, j, c=c: oracle.mul(c["x0"][i:j], c["x1"][i:j], c["y0"][i:j], c["y1"][i:j]),
            lambda i, j, c=c: oracle.div(c["x0"][i:j], c["x1"][i:j], c["y0"][i:j], c["y1"][i:j]),
            lambda i, j, s=s: oracle.sqrt(s["x0"][i:j], s["x1"][i:j]),
            lambda i, j, c=c, a=a: oracle.axpy(a, c["x0"][i:j], c["x1"][i:j], c["y0"][i:j], c["y1"][i:j]),
            lambda i, j, h=h: oracle.horner(h["c"], h["x0"][i:j], h["x1"][i:j]),
            lambda i, j, hi=hi, lo=lo: oracle.sum(hi[i:j], lo[i:j]),
            lambda i, j, r=r: oracle.dot(r["x"][i:j], None, r["y"][i:j], None),
        ])
    jobs = [j for js in jobs_by_type for j in js]

    def timed(run, budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            for job in jobs:
                run(job)
            reps += 1
            if time.perf_counter() - t0 > budget:
                return reps * n * len(jobs), time.perf_counter() - t0

    e1, t1 = timed(lambda job: job(0, n), seconds_target)
    chunk = n // cores
    bounds = [(k * chunk, n if k == cores - 1 else (k + 1) * chunk) for k in range(cores)]
    with ThreadPoolExecutor(cores) as pool:
        ea, ta = timed(lambda job: list(pool.map(lambda b: job(*b), bounds)), seconds_target / 3)
    return {"value": ea / ta / 1e9, "unit": "Gelem/s", "cores": cores, "kind": "oracle",
            "value_1_thread": e1 / t1 / 1e9,
            "sample": "every kernel of the step (add, sub, mul, div, sqrt, axpy, horner-8, sum, dot), "
                      "binary64 and binary32, on n = 2^20 elements each: %.1f s on 1 thread, then %.1f s "
                      "partitioned over %d threads" % (t1, ta, cores)}


def serving_run(torch, W, jobs=20000, rate=2000.0, budget=64 << 30, seed=1):
    """The verification-job stream on the persistent kernel: Poisson
    arrivals, sum / dot / axpy / Horner-8 of log-uniform lengths 2^8 .. 2^24,
    half binary32, 5 % ill-conditioned (sum / dot: instances of the
    ill-conditioned dot generator at condition number 1e20, uploaded before
    the clock starts, length rounded to a power of two; axpy / Horner:
    cancelling inputs generated on the device).  Latency = completion seen
    by the host - scheduled arrival."""
    import numpy as np
    from paper_1401_6235_amd import serve as S

    sched = W.serve_schedule(jobs, rate, seed=seed)
    # ill-conditioned instances, one per (length, dtype, op)
    inst = {}
    for j in sched:
        if j["illcond"] and j["op"] in ("sum", "dot"):
            n2 = 1 << int(round(np.log2(j["n"])))
            n2 = min(max(n2, 256), 1 << 24)
            j["n"] = n2
            inst.setdefault((n2, j["dtype"]), None)
    log("serving: generating %d ill-conditioned instances" % len(inst))
    dev = "cuda"
    for (n2, dt) in sorted(inst):
        npdt = np.float64 if dt == "f64" else np.float32
        d = W.illdot_case(n2, 1e20, seed=n2, dtype=npdt)
        hi, lo = W.product_split(d["x"], d["y"])
        inst[(n2, dt)] = {k: torch.from_numpy(v).to(dev) for k, v in
                          (("x", d["x"]), ("y", d["y"]), ("hi", hi), ("lo", lo))}

    def job_of(j):
        if j["illcond"] and j["op"] in ("sum", "dot"):
            t = inst[(j["n"], j["dtype"])]
            if j["op"] == "dot":
                return S.make_job("dot", j["dtype"], j["n"], kind=S.TFS_KIND_PROVIDED, x0=t["x"], y0=t["y"])
            return S.make_job("sum", j["dtype"], j["n"], kind=S.TFS_KIND_PROVIDED, x0=t["hi"], x1=t["lo"])
        kind = S.TFS_KIND_ILLCOND if j["illcond"] else S.TFS_KIND_RANDOM
        c = (W.HORNER_ILLCOND_C if j["illcond"] else j["c"]) if j["op"] == "horner" else None
        return S.make_job(j["op"], j["dtype"], j["n"], seed=j["seed"], kind=kind, c=c)

    descs = [job_of(j) for j in sched]
    torch.cuda.synchronize()
    srv = S.Server(0, budget, S.TFS_MAX_SLOTS)
    try:
        log("serving: %d jobs at %.0f jobs/s" % (jobs, rate))
        ids, results = S.run_stream(srv, [j["t"] for j in sched], descs)
        stats = srv.stats()
    finally:
        srv.close()
    res = [results[i] for i in ids if i in results]
    lat = np.array([r["t_done"] - r["t_arrive"] for r in res])
    span = max(r["t_done"] for r in res) - min(r["t_arrive"] for r in res)
    elems = sum(r["n"] for r in res)
    flags = {}
    agree = {"illcond_flagged": 0, "illcond": 0, "random_flagged": 0, "random": 0}
    for j, i in zip(sched, ids):
        r = results.get(i)
        if r is None:
            continue
        key = "%s_%s%s" % (j["op"], j["dtype"], "_ill" if j["illcond"] else "")
        f = flags.setdefault(key, [0, 0])
        f[0] += 1
        f[1] += r["flag"]
        if j["illcond"]:
            agree["illcond"] += 1
            agree["illcond_flagged"] += r["flag"]
        else:
            agree["random"] += 1
            agree["random_flagged"] += r["flag"]
    def pct(xs, q):
        return round(float(np.percentile(np.array(xs), q)) * 1e6, 1)

    stages = {
        "submit_late": [r["t_submit"] - r["t_arrive"] for r in res],
        "admit": [r["t_admit"] - r["t_submit"] for r in res],
        "publish": [r["t_publish"] - r["t_admit"] for r in res],
        "device_and_completion": [r["t_done"] - r["t_publish"] for r in res],
        # inside device_and_completion, from the device clock: slot opened to
        # first unit claimed, input generation, compute units to the record
        "device_queue": [r["queue_us"] * 1e-6 for r in res],
        "device_gen": [r["gen_us"] * 1e-6 for r in res],
        "device_run": [r["device_us"] * 1e-6 for r in res],
    }
    breakdown = {"%s_us_p%d" % (k, q): pct(v, q) for q in (50, 99) for k, v in stages.items()}
    return {
        "jobs": jobs, "completed": len(res), "rate_offered": rate,
        "latency_breakdown": breakdown,
        "p50_us": round(float(np.percentile(lat, 50)) * 1e6, 1),
        "p99_us": round(float(np.percentile(lat, 99)) * 1e6, 1),
        "mean_us": round(float(lat.mean()) * 1e6, 1),
        "jobs_per_s": round(len(res) / span, 1),
        "gelem_s": round(elems / span / 1e9, 3),
        "device_us_p50": round(float(np.percentile([r["device_us"] for r in res], 50)), 1),
        "peak_resident_gib": round(stats["peak_resident_bytes"] / 2 ** 30, 3),
        "budget_gib": budget / 2 ** 30,
        "admission_waits": stats["admission_waits"],
        "flags_by_job": {k: {"jobs": v[0], "flagged": v[1]} for k, v in sorted(flags.items())},
        "flag_summary": agree,
        "status_ok": all(r["status"] == 0 for r in res),
    }


# ---------------------------------------------------------------------------
# In-register regime (the paper's "data in cache" criterion) and the batched
# applications
# ---------------------------------------------------------------------------

CHAIN_N = 1 << 21
CHAIN_REPS = 2048
FP_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # MI355X vector FP64 / FP32, published
# Algorithmic floating-point operations of one chain step, counting each
# + - * / sqrt as one and each fma as two (the convention of the peaks).
# TS = 6, TP = 3 (a multiply and an fma), Fast Two-Sum = 3.
STEP_FLOPS = {
    ("add", "twofold", True): 8, ("add", "twofold", False): 7,
    ("sub", "twofold", True): 8, ("sub", "twofold", False): 7,
    ("mul", "twofold", True): 9, ("mul", "twofold", False): 5,
    ("div", "twofold", True): 8, ("div", "twofold", False): 5,
    ("sqrt", "twofold", True): 21,
    ("add", "coupled", True): 8, ("sub", "coupled", True): 8, ("mul", "coupled", True): 7,
    ("div", "coupled", True): 7, ("sqrt", "coupled", True): 6,
}
TRSV_NSYS, TRSV_M = 1 << 20, 16           # dense 16 x 16 systems
JORDAN_NSYS, JORDAN_M = 1 << 24, 3         # the paper's 3 x 3 Jordan blocks
QUAD_N = 1 << 24
FMA_N = 1 << 26


def time_call(torch, fn, steps, warmup):
    """Average HIP-event duration (ms) of fn() on the current stream."""
    for _ in range(warmup):
        fn()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / steps


def in_register_run(torch, tf, W, steps=3, warmup=1):
    """Chains of CHAIN_REPS steps on CHAIN_N elements held in registers:
    twofold (twofold and dotted operand), coupled and Dekker mode against
    the plain chain.  The paper's criterion is twofold/plain <= 10 here."""
    import numpy as np
    out = {"n": CHAIN_N, "reps": CHAIN_REPS, "ops": {}}
    for dt, tag in ((np.float64, "f64"), (np.float32, "f32")):
        for op in ("add", "sub", "mul", "div", "sqrt"):
            c = W.chain_case(op, CHAIN_N, seed=0, dtype=dt)
            g = {k: torch.from_numpy(v).cuda() for k, v in c.items()}
            z0, z1 = torch.empty_like(g["x0"]), torch.empty_like(g["x0"])
            y0, y1 = g.get("y0"), g.get("y1")
            plain = time_call(torch, lambda: tf.tf_plain_chain(op, CHAIN_REPS, g["x0"], y0, z0), steps, warmup)
            row = {"plain_ms": round(plain, 4)}
            variants = [("twofold", True), ("coupled", True), ("dekker", True)]
            if op != "sqrt":
                variants.insert(1, ("twofold", False))
            for mode, yt in variants:
                ms = time_call(torch, lambda: tf.tf_chain(op, mode, CHAIN_REPS, g["x0"], g["x1"], y0,
                                                          y1 if yt else None, z0, z1), steps, warmup)
                key = mode if yt else mode + "_dotted_y"
                flops = STEP_FLOPS.get((op, "coupled" if mode == "dekker" else mode, yt))
                if flops is not None and mode == "dekker":
                    flops += 3
                steps_s = CHAIN_N * CHAIN_REPS / (ms * 1e-3)
                row[key] = {"ms": round(ms, 4), "gop_s": round(steps_s / 1e9, 1),
                            "slowdown": round(ms / plain, 2)}
                if flops is not None:
                    tfl = flops * steps_s / 1e12
                    row[key]["tflop_s"] = round(tfl, 2)
                    row[key]["frac_fp_peak"] = round(tfl / FP_PEAK_TFLOPS[tag], 4)
            row["plain_gop_s"] = round(CHAIN_N * CHAIN_REPS / (plain * 1e-3) / 1e9, 1)
            out["ops"]["%s_%s" % (op, tag)] = row
            del g, z0, z1
    worst = max(v["twofold"]["slowdown"] for v in out["ops"].values())
    out["max_twofold_slowdown"] = worst
    out["meets_10x"] = worst <= 10.0
    return out


def applications_run(torch, tf, W, steps=3, warmup=1):
    """Batched back-substitution (the paper's 3 x 3 Jordan blocks, 2^24
    systems; dense 16 x 16, 2^20 systems), both quadratic roots (n = 2^24)
    and the twofold fma
    (n = 2^26): time, HBM rate of the algorithmic bytes, slowdown against
    the plain kernels."""
    import numpy as np
    out = {}
    for dt, tag, es in ((np.float64, "f64", 8), (np.float32, "f32", 4)):
        for key, kind, m, ns in (("jordan3", "jordan", JORDAN_M, JORDAN_NSYS), ("trsv16", "dense", TRSV_M, TRSV_NSYS)):
            c = W.trsv_case(m, ns, seed=0, dtype=dt, kind=kind)
            g = {k: torch.from_numpy(v).cuda() for k, v in c.items() if k != "m"}
            del c
            x0, x1 = torch.empty_like(g["f0"]), torch.empty_like(g["f0"])
            ms = time_call(torch, lambda: tf.tf_trsv_upper(m, g["U0"], g["U1"], g["f0"], g["f1"], x0, x1),
                           steps, warmup)
            pms = time_call(torch, lambda: tf.tf_plain_trsv_upper(m, g["U0"], g["f0"], x0), steps, warmup)
            alg = (m * (m + 1) // 2 * 2 + 4 * m) * es * ns  # upper U twofold, f and x twofold
            palg = (m * (m + 1) // 2 + 2 * m) * es * ns
            out["%s_%s" % (key, tag)] = {
                "nsys": ns, "m": m, "ms": round(ms, 4), "plain_ms": round(pms, 4),
                "gb_s": round(alg / ms / 1e6, 1), "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4),
                "plain_gb_s": round(palg / pms / 1e6, 1), "slowdown": round(ms / pms, 3)}
            del g, x0, x1
        q = W.quadratic_case(QUAD_N, seed=0, dtype=dt)
        g = {k: torch.from_numpy(v).cuda() for k, v in q.items()}
        outs = tuple(torch.empty_like(g["a0"]) for _ in range(4))
        keys = ("a0", "a1", "b0", "b1", "c0", "c1")
        ms = time_call(torch, lambda: tf.tf_quadratic(*[g[k] for k in keys], out=outs), steps, warmup)
        pms = time_call(torch, lambda: tf.tf_plain_quadratic(g["a0"], g["b0"], g["c0"], outs[0], outs[1]),
                        steps, warmup)
        alg = 10 * es * QUAD_N
        out["quadratic_" + tag] = {"n": QUAD_N, "ms": round(ms, 4), "plain_ms": round(pms, 4),
                                   "gb_s": round(alg / ms / 1e6, 1),
                                   "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4),
                                   "slowdown": round(ms / pms, 3)}
        del g, outs
        f = W.fma_case(FMA_N, seed=0, dtype=dt)
        g = {k: torch.from_numpy(v).cuda() for k, v in f.items()}
        del f
        z0, z1 = torch.empty_like(g["x0"]), torch.empty_like(g["x0"])
        keys = ("x0", "x1", "y0", "y1", "w0", "w1")
        ms = time_call(torch, lambda: tf.tf_fma(*[g[k] for k in keys], z0, z1), steps, warmup)
        pms = time_call(torch, lambda: tf.tf_plain_fma(g["x0"], g["y0"], g["w0"], z0), steps, warmup)
        alg = 8 * es * FMA_N
        out["fma_" + tag] = {"n": FMA_N, "ms": round(ms, 4), "plain_ms": round(pms, 4),
                             "gb_s": round(alg / ms / 1e6, 1), "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4),
                             "slowdown": round(ms / pms, 3)}
        del g, z0, z1
        torch.cuda.empty_cache()
    return out


# rocprofv3 kernel names -> bench keys
_OPS = {"0": "add", "1": "sub", "2": "mul", "3": "div", "4": "sqrt"}
_CHAIN = {0: "add", 1: "sub", 2: "mul", 3: "div", 4: "sqrt", 5: "mul_coupled", 6: "div_coupled",
          7: "sqrt_coupled", 8: "add_dekker", 9: "sub_dekker", 13: "mul_dekker", 14: "div_dekker",
          15: "sqrt_dekker"}


def bench_key(name: str):
    import re
    t = "f64" if "<double" in name else "f32" if "<float" in name else None
    if t is None:
        return None
    m = re.search(r"ew_vec_kernel<\w+, (\d), true, (true|false)", name)
    # both operands twofold (the square root: its one operand); the dotted
    # forms timed outside the step launch the same kernels' other variants
    if m and m.group(1) in _OPS and (m.group(2) == "true") == (m.group(1) != "4"):
        return "%s_%s" % (_OPS[m.group(1)], t)
    if "axpy_vec_kernel" in name and "true, true" in name:
        return "axpy_" + t
    if re.search(r"\bhorner_kernel<\w+, true>", name):
        return "horner_" + t
    m = re.search(r"reduce_tiles_kernel<\w+, (\d),", name)
    if m and m.group(1) in ("1", "2"):
        return ("sum_" if m.group(1) == "1" else "dot_") + t
    if re.search(r"plain_vec_kernel<\w+, 99,", name):
        return "vmem_" + t
    m = re.search(r"\bchain_kernel<\w+, (\d+), (true|false)", name)
    if m and "plain_chain" not in name:
        code, yt = int(m.group(1)), m.group(2) == "true"
        op = _CHAIN.get(code)
        if op is None:
            return None
        return "chain_%s%s_%s" % (op, "" if yt or "sqrt" in op else "_dotted_y", t)
    m = re.search(r"plain_chain_kernel<\w+, (\d),", name)
    if m:
        return "plain_chain_%s_%s" % (_OPS[m.group(1)], t)
    m = re.search(r"\btrsv_fixed_kernel<\w+, (\d+), true, true>", name)
    if m and "plain" not in name:
        return {"3": "jordan3_", "16": "trsv16_"}.get(m.group(1), "trsv%s_" % m.group(1)) + t
    m = re.search(r"plain_trsv_fixed_kernel<\w+, (\d+)>", name)
    if m:
        return "plain_" + {"3": "jordan3_", "16": "trsv16_"}.get(m.group(1), "trsv%s_" % m.group(1)) + t
    if "quadratic_vec_kernel" in name:
        return "quadratic_" + t
    if "plain_quadratic_kernel" in name:
        return "plain_quadratic_" + t
    if "fma_vec_kernel" in name and "true, true, true" in name:
        return "fma_" + t
    if "plain_fma_kernel" in name:
        return "plain_fma_" + t
    return None


def alg_bytes(key: str):
    """Algorithmic HBM bytes of one launch of a benchmarked kernel."""
    base, t = key.rsplit("_", 1)
    es = 8 if t == "f64" else 4
    plain = base.startswith("plain_")
    b = base[6:] if plain else base
    if b == "vmem":
        return 3 * es * N_STREAM
    if plain and base in PLAIN_WORDS:
        return PLAIN_WORDS[base] * es * (N_REDUCE if b in ("sum", "dot") else N_STREAM)
    if b in KERNELS:
        n = N_REDUCE if b in ("sum", "dot") else N_STREAM
        return KERNELS[b][0] * es * n
    if b in ("jordan3", "trsv16"):
        m, ns = (JORDAN_M, JORDAN_NSYS) if b == "jordan3" else (TRSV_M, TRSV_NSYS)
        words = (m * (m + 1) // 2 + 2 * m) if plain else (m * (m + 1) // 2 * 2 + 4 * m)
        return words * es * ns
    if b == "quadratic":
        return (5 if plain else 10) * es * QUAD_N
    if b == "fma":
        return (4 if plain else 8) * es * FMA_N
    return None


_GROUPS = [
    ("hot_path_step_n2e28", "the benchmark step (n = 2^28 elementwise, 2^26 reductions)",
     lambda k: k.rsplit("_", 1)[0] in KERNELS or k.startswith("vmem")),
    ("chains_n2e21_reps2048", "the in-register chains (n = 2^21, 2048 steps)",
     lambda k: k.startswith("chain_") or k.startswith("plain_chain_")),
    ("applications_jordan3_trsv16_quadratic_fma",
     "the batched applications (3x3 Jordan 2^24, 16x16 dense 2^20, quadratic 2^24, fma 2^26)",
     lambda k: k.rsplit("_", 1)[0].replace("plain_", "") in ("jordan3", "trsv16", "quadratic", "fma")),
]


def _bench_dispatches(rows, name_col, grid_col):
    """Per bench key, the dispatch rows at that kernel's largest grid: the
    benchmark's own launches (the cache-resident leg launches some of the
    same kernels over far smaller grids)."""
    acc = {}
    for r in rows:
        k = bench_key(r[name_col])
        if k:
            acc.setdefault(k, []).append(r)
    out = {}
    for k, rs in acc.items():
        g = max(int(r[grid_col]) for r in rs)
        out[k] = (g, [r for r in rs if int(r[grid_col]) == g])
    return out


def summarize_profiles(prof_dir: str, command: str, out_dir: str = None):
    """Write profiles/<group>_kernel_trace.txt, <group>_counters.txt and
    profiles/traffic.json from rocprofv3 runs of this benchmark: kernel
    statistics (--kernel-trace --stats) in prof_dir/trace, FETCH_SIZE and
    WRITE_SIZE (--pmc, one counter per run) in prof_dir/fetch and
    prof_dir/write.  FETCH_SIZE / WRITE_SIZE are scaled by the factor that
    makes them equal the known bytes of the copy kernel (vmem)."""
    import csv
    import glob
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    trace = glob.glob(os.path.join(prof_dir, "trace", "*kernel_trace.csv"))[0]
    disp = _bench_dispatches(csv.DictReader(open(trace)), "Kernel_Name", "Grid_Size_X")
    rows = []  # one per bench key: the launches at the benchmark's own (largest) grid
    for k, (grid, ds) in disp.items():
        span = [(float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) for r in ds]
        rows.append({"key": k, "Name": ds[0]["Kernel_Name"], "Calls": len(ds), "grid": grid,
                     "AverageNs": sum(span) / len(span), "TotalDurationNs": sum(span)})
    src = kernel_source_hash()
    for fname, what, member in _GROUPS:
        lines = ["# rocprofv3 kernel statistics of " + what,
                 "# command: " + command, "# source hash: " + src,
                 "# (launches at the benchmark's grid only: the same kernels' smaller launches of the",
                 "# cache-resident leg, n = 2^20, are left out)",
                 "%-28s %6s %12s %11s  %s" % ("bench_key", "calls", "avg_us", "grid", "kernel")]
        for r in sorted(rows, key=lambda r: -r["TotalDurationNs"]):
            if member(r["key"]):
                lines.append("%-28s %6d %12.2f %11d  %s" % (r["key"], r["Calls"], r["AverageNs"] / 1e3, r["grid"],
                                                            r["Name"][:100]))
        open(os.path.join(out_dir, fname + "_kernel_trace.txt"), "w").write("\n".join(lines) + "\n")

    def counters(which):
        f = glob.glob(os.path.join(prof_dir, which, "*counter_collection.csv"))[0]
        d = _bench_dispatches(csv.DictReader(open(f)), "Kernel_Name", "Grid_Size")
        return {k: sum(float(r["Counter_Value"]) for r in ds) / len(ds) for k, (_, ds) in d.items()}

    fetch, write = counters("fetch"), counters("write")
    traffic = {"source_hash": src, "command": command, "kernels": {}}
    factors = {}
    for t, es in (("f64", 8), ("f32", 4)):
        n = N_STREAM
        f = (2 * n * es) / (fetch["vmem_" + t] * 1024)
        w = (n * es) / (write["vmem_" + t] * 1024)
        factors[t] = (f, w)
    traffic["scale"] = {t: {"fetch": round(f, 4), "write": round(w, 4)} for t, (f, w) in factors.items()}
    for fname, what, member in _GROUPS:
        keys = [k for k in sorted(set(fetch) & set(write)) if member(k) and alg_bytes(k)]
        if not keys or fname.startswith("chains"):
            continue
        lines = ["# HBM traffic per launch of " + what + ", from rocprofv3 --pmc FETCH_SIZE and",
                 "# --pmc WRITE_SIZE (KiB per dispatch, one counter per run), scaled so the copy kernel",
                 "# reads and writes its known bytes",
                 "# command: " + command, "# source hash: " + src,
                 "# scale factors (fetch, write): " + json.dumps(traffic["scale"]),
                 "%-24s %14s %14s %16s %16s %8s" % ("bench_key", "FETCH_KiB", "WRITE_KiB", "traffic_B",
                                                    "algorithmic_B", "ratio")]
        for k in keys:
            t = k.rsplit("_", 1)[1]
            f, w = factors[t]
            b = fetch[k] * 1024 * f + write[k] * 1024 * w
            alg = alg_bytes(k)
            traffic["kernels"][k] = {"fetch_kib": fetch[k], "write_kib": write[k], "bytes_per_launch": round(b),
                                     "algorithmic_bytes": alg}
            lines.append("%-24s %14.0f %14.0f %16.0f %16d %8.4f" % (k, fetch[k], write[k], b, alg, b / alg))
        open(os.path.join(out_dir, fname + "_counters.txt"), "w").write("\n".join(lines) + "\n")
        print("\n".join(lines))
    json.dump(traffic, open(os.path.join(out_dir, "traffic.json"), "w"), indent=1)
    if os.path.isdir(os.path.join(prof_dir, "valu64")) and os.path.isdir(os.path.join(prof_dir, "valu32")):
        summarize_valu(prof_dir, command, rows, out_dir)
    summarize_memory(prof_dir, command, out_dir)


# Memory-pipeline counter sets (one rocprofv3 --pmc run each, directories
# mem1 .. mem5), within the per-block limits of one pass.
MEM_SETS = [
    "TCC_EA0_RDREQ_sum TCC_EA0_WRREQ_sum TCC_EA0_RDREQ_DRAM_CREDIT_STALL_sum TCC_EA0_WRREQ_DRAM_CREDIT_STALL_sum",
    "TCC_TAG_STALL_sum TCC_TOO_MANY_EA_WRREQS_STALL_sum TCC_EA0_WRREQ_64B_sum TCC_EA0_RDREQ_128B_sum",
    "TCP_TCC_READ_REQ_LATENCY_sum TCP_TCC_READ_REQ_sum TCP_TCC_WRITE_REQ_LATENCY_sum TCP_TCC_WRITE_REQ_sum",
    "TA_BUSY_avr TA_ADDR_STALLED_BY_TC_CYCLES_sum TD_TC_STALL_sum TD_TD_BUSY_sum TCP_UTCL1_TRANSLATION_MISS_sum "
    "TCP_PENDING_STALL_CYCLES_sum TCP_TCR_TCP_STALL_CYCLES_sum GRBM_GUI_ACTIVE",
    "SQ_WAIT_ANY SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_WAVES SQ_INST_LEVEL_VMEM "
    "SQ_WAIT_INST_ANY",
]


def summarize_memory(prof_dir: str, command: str, out_dir: str = None):
    """profiles/hot_path_step_n2e28_memory_counters.txt from the MEM_SETS
    runs: per streaming kernel of the step, requests to HBM, the L1's
    average read / write latency to the L2, stalls of the texture addresser
    by the L1, L2 tag stalls, DRAM credit stalls and address-translation
    misses, each per KiB moved, and the kernel's cycles per MiB."""
    import csv
    import glob
    acc = {}
    for i in range(1, len(MEM_SETS) + 1):
        f = glob.glob(os.path.join(prof_dir, "mem%d" % i, "*counter_collection.csv"))
        if not f:
            return
        for k, (_, ds) in _bench_dispatches(csv.DictReader(open(f[0])), "Kernel_Name", "Grid_Size").items():
            for r in ds:
                acc.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    c = {k: {n: sum(v) / len(v) for n, v in d.items()} for k, d in acc.items()}
    keys = [k for k in ("add_f64", "sub_f64", "mul_f64", "div_f64", "axpy_f64", "vmem_f64",
                        "add_f32", "sub_f32", "mul_f32", "div_f32", "axpy_f32", "vmem_f32") if k in c]
    lines = ["# Memory pipeline of the step's streaming kernels (n = 2^28), from rocprofv3 --pmc runs of",
             *["#   " + m for m in MEM_SETS],
             "# per dispatch: cycles per MiB moved (GRBM_GUI_ACTIVE), HBM read / write requests per KiB,",
             "# average L1 -> L2 read and write latency in cycles, and per KiB: texture-addresser cycles",
             "# stalled by the L1, L2 tag stalls, DRAM read / write credit stalls, address-translation misses",
             "# command: " + command, "# source hash: " + kernel_source_hash(),
             "%-10s %9s %7s %7s %8s %8s %9s %8s %8s %8s %8s" % (
                 "bench_key", "cyc/MiB", "rd/KiB", "wr/KiB", "rd_lat", "wr_lat", "ta_stall", "tag_stl",
                 "dram_rd", "dram_wr", "tlb_miss")]
    for k in keys:
        d = c[k]
        kib = alg_bytes(k) / 1024.0
        g = lambda n: d.get(n, float("nan"))
        lines.append("%-10s %9.0f %7.3f %7.3f %8.0f %8.0f %9.4f %8.4f %8.4f %8.4f %8.5f" % (
            k, g("GRBM_GUI_ACTIVE") / (kib / 1024.0), g("TCC_EA0_RDREQ_sum") / kib, g("TCC_EA0_WRREQ_sum") / kib,
            g("TCP_TCC_READ_REQ_LATENCY_sum") / g("TCP_TCC_READ_REQ_sum"),
            g("TCP_TCC_WRITE_REQ_LATENCY_sum") / g("TCP_TCC_WRITE_REQ_sum"),
            g("TA_ADDR_STALLED_BY_TC_CYCLES_sum") / kib, g("TCC_TAG_STALL_sum") / kib,
            g("TCC_EA0_RDREQ_DRAM_CREDIT_STALL_sum") / kib, g("TCC_EA0_WRREQ_DRAM_CREDIT_STALL_sum") / kib,
            g("TCP_UTCL1_TRANSLATION_MISS_sum") / kib))
    out = os.path.join(out_dir or os.path.join(ROOT, "profiles"), "hot_path_step_n2e28_memory_counters.txt")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


VALU64 = "SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64 " \
         "SQ_ACTIVE_INST_VALU SQ_INSTS_VALU GRBM_GUI_ACTIVE"
VALU32 = "SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_TRANS_F32 " \
         "SQ_THREAD_CYCLES_VALU GRBM_GUI_ACTIVE"


def summarize_valu(prof_dir: str, command: str, trace_rows, out_dir: str = None):
    """profiles/<group>_valu.txt from two --pmc runs (VALU64, VALU32
    counters) of the benchmark: executed FP64 / FP32 operations per launch
    (each ADD / MUL / TRANS wave instruction is 64 operations, each FMA 128)
    and their rate over the kernel's average traced duration against the
    vector peaks (78.6 / 157.3 TFLOP/s); VALU wave instructions per CU per
    cycle (SQ_INSTS_VALU over the counted run's cycles: GRBM_GUI_ACTIVE,
    summed over the 8 XCDs, divided by 8) and the clock of that run (cycles
    over its own dispatch duration)."""
    import csv
    import glob
    dur = {r["key"]: r["AverageNs"] * 1e-9 for r in trace_rows}

    def per_kernel(which):
        f = glob.glob(os.path.join(prof_dir, which, "*counter_collection.csv"))[0]
        acc, span = {}, {}
        for k, (_, ds) in _bench_dispatches(csv.DictReader(open(f)), "Kernel_Name", "Grid_Size").items():
            for r in ds:
                acc.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                span.setdefault(k, {})[r["Dispatch_Id"]] = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9
        out = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}
        for k, d in span.items():
            out[k]["_seconds"] = sum(d.values()) / len(d)
        return out

    c64, c32 = per_kernel("valu64"), per_kernel("valu32")
    src = kernel_source_hash()
    for fname, what, member in _GROUPS:
        keys = [k for k in sorted(set(c64) & set(c32) & set(dur)) if member(k)]
        if not keys:
            continue
        lines = ["# VALU work per launch of " + what + ", from rocprofv3 --pmc runs of",
                 "# " + VALU64, "# and " + VALU32,
                 "# (per dispatch; FP ops = 64 per ADD/MUL/TRANS wave instruction, 128 per FMA; TFLOP/s over the",
                 "# traced average duration against the peaks 78.6 (FP64) / 157.3 (FP32); valu_ipc = SQ_INSTS_VALU",
                 "# per CU per cycle, cycles = GRBM_GUI_ACTIVE / 8 XCDs; issue ceiling 1.0 for full-rate FP64",
                 "# instructions (4 SIMDs x one wave instruction per 4 cycles) and 2.0 for FP32, which issues at",
                 "# twice that rate (the FP32 chains reach 1.8); GHz = cycles / the counted dispatch's own",
                 "# duration, an estimate that short dispatches overstate by a few percent)",
                 "# command: " + command, "# source hash: " + src,
                 "%-28s %10s %12s %8s %12s %8s %9s %6s" % ("bench_key", "avg_us", "fp64_TFLOP/s", "frac64",
                                                        "fp32_TFLOP/s", "frac32", "valu_ipc", "GHz")]
        for k in keys:
            a, b = c64[k], c32[k]
            t = dur[k]
            f64 = 64 * (a.get("SQ_INSTS_VALU_ADD_F64", 0) + a.get("SQ_INSTS_VALU_MUL_F64", 0)
                        + a.get("SQ_INSTS_VALU_TRANS_F64", 0) + 2 * a.get("SQ_INSTS_VALU_FMA_F64", 0))
            f32 = 64 * (b.get("SQ_INSTS_VALU_ADD_F32", 0) + b.get("SQ_INSTS_VALU_MUL_F32", 0)
                        + b.get("SQ_INSTS_VALU_TRANS_F32", 0) + 2 * b.get("SQ_INSTS_VALU_FMA_F32", 0))
            cycles = a.get("GRBM_GUI_ACTIVE", 0) / 8
            ipc = a.get("SQ_INSTS_VALU", 0) / (cycles * 256) if cycles else 0
            ghz = cycles / a["_seconds"] / 1e9 if a.get("_seconds") else 0
            lines.append("%-28s %10.1f %12.2f %8.4f %12.2f %8.4f %9.3f %6.2f" % (
                k, t * 1e6, f64 / t / 1e12, f64 / t / 1e12 / FP_PEAK_TFLOPS["f64"], f32 / t / 1e12,
                f32 / t / 1e12 / FP_PEAK_TFLOPS["f32"], ipc, ghz))
        open(os.path.join(out_dir or os.path.join(ROOT, "profiles"), fname + "_valu.txt"), "w").write(
            "\n".join(lines) + "\n")
        print("\n".join(lines))



CACHE_N = 1 << 20
CACHE_LAUNCHES = 50


def cache_resident_run(torch, tf, W, warmup=3):
    """The paper's "medium" arrays (its L3 case): elementwise operations at
    n = 2^20, whose operands (at most 48 MiB in binary64) stay in the 256 MB
    Infinity Cache across back-to-back calls.  Time of CACHE_LAUNCHES calls
    in a row between two HIP events, per call; twofold (both operands
    twofold) against plain."""
    import numpy as np
    out = {"n": CACHE_N, "launches": CACHE_LAUNCHES, "ops": {}}
    stream = torch.cuda.current_stream()
    for dt, tag, es in ((np.float64, "f64", 8), (np.float32, "f32", 4)):
        for op in ("add", "sub", "mul", "div", "sqrt"):
            c = W.elementwise(op, CACHE_N, seed=0, dtype=dt)
            g = {k: torch.from_numpy(v).cuda() for k, v in c.items()}
            z0, z1 = torch.empty_like(g["x0"]), torch.empty_like(g["x0"])
            if op == "sqrt":
                two = lambda: tf.tf_sqrt(g["x0"], g["x1"], z0, z1)  # noqa: E731
                one = lambda: tf.tf_plain_sqrt(g["x0"], z0)  # noqa: E731
                words = (4, 2)
            else:
                two = lambda: getattr(tf, "tf_" + op)(g["x0"], g["x1"], g["y0"], g["y1"], z0, z1)  # noqa: E731
                one = lambda: getattr(tf, "tf_plain_" + op)(g["x0"], g["y0"], z0)  # noqa: E731
                words = (6, 3)
            res = []
            for fn in (two, one):
                for _ in range(warmup):
                    fn()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(CACHE_LAUNCHES):
                    fn()
                b.record(stream)
                torch.cuda.synchronize()
                res.append(a.elapsed_time(b) / CACHE_LAUNCHES)
            ms, pms = res
            out["ops"]["%s_%s" % (op, tag)] = {
                "ms": round(ms, 5), "gelem_s": round(CACHE_N / ms / 1e6, 1),
                "gb_s": round(words[0] * es * CACHE_N / ms / 1e6, 1), "plain_ms": round(pms, 5),
                "plain_gelem_s": round(CACHE_N / pms / 1e6, 1), "slowdown": round(ms / pms, 3)}
            del g, z0, z1
    return out


# The paper's own twofold/plain ratios (its Tables 1 and 2: Intel Core
# i5-4200U, AVX2, binary64, both operands twofold; sub against vadd, as the
# paper has no vsub): large arrays (DRAM) and small ones (L1).
PAPER_SLOWDOWN_LARGE = {"add": 2.10, "sub": 2.17, "mul": 2.04, "div": 2.22, "sqrt": 3.41}
PAPER_SLOWDOWN_SMALL = {"add": 6.48, "sub": 6.59, "mul": 3.95, "div": 2.23, "sqrt": 3.35}


PAPER_SLOWDOWN_MEDIUM = {"add": 2.04, "sub": 2.10, "mul": 2.00, "div": 2.23, "sqrt": 3.37}


# The paper's Tables 1-2, large arrays, binary64 (Mflop/s): plain operations
# and the twofold ones with one dotted operand (*1) or two (exact
# transforms; for sqrt, the dotted argument, RPF1.1).  vsub is not listed:
# vadd stands in for it.
PAPER_PLAIN_LARGE_F64 = {"add": 484.135, "sub": 484.135, "mul": 485.604, "div": 356.078, "sqrt": 361.607}
PAPER_ONE_DOTTED_LARGE_F64 = {"add": 259.465, "sub": 263.608, "mul": 279.025, "div": 160.605}
PAPER_BOTH_DOTTED_LARGE_F64 = {"add": 306.501, "sub": 329.568, "mul": 331.331, "div": 158.014, "sqrt": 160.645}


def dotted_forms_run(torch, tf, inputs, pper, steps, warmup):
    """The dotted and mixed operand forms at n = 2^28: one operand dotted
    (ATF1.1, STF1.1, MTF1.1, DTF1.1 with y dotted; the x-dotted forms), both
    dotted (the exact transforms Two-Sum, Two-Diff, Two-Product and DTF1.1.1)
    and the dotted square root (RPF1.1), each against the plain kernel of the
    same operation timed in the plain pass."""
    calls, words = [], {}
    for key, d in inputs.items():
        tag = "f64" if key == "float64" else "f32"
        z0, z1 = d["z0"], d["z1"]
        for op in ("add", "sub", "mul", "div"):
            f = getattr(tf, "tf_" + op)
            forms = (("y_dotted", lambda f=f, d=d, z0=z0, z1=z1: f(d["x0"], d["x1"], d["y0"], None, z0, z1), 5),
                     ("x_dotted", lambda f=f, d=d, z0=z0, z1=z1: f(d["x0"], None, d["y0"], d["y1"], z0, z1), 5),
                     ("both_dotted", lambda f=f, d=d, z0=z0, z1=z1: f(d["x0"], None, d["y0"], None, z0, z1), 4))
            for form, fn, w in forms:
                name = "%s_%s_%s" % (op, form, tag)
                calls.append((name, N_STREAM, fn))
                words[name] = w
        name = "sqrt_dotted_%s" % tag
        calls.append((name, N_STREAM, lambda d=d, z0=z0, z1=z1: tf.tf_sqrt(d["s0"], None, z0, z1)))
        words[name] = 3
    _, per = run_pass(torch, calls, steps, warmup)
    out = {}
    for name, n, _ in calls:
        op, tag = name.split("_", 1)[0], name.rsplit("_", 1)[1]
        es = 8 if tag == "f64" else 4
        ms = per[name]["ms_avg"]
        p = pper["plain_%s_%s" % (op, tag)]["ms_avg"]
        v = pper["vmem_" + tag]["ms_avg"]
        gbs = n * words[name] * es / ms / 1e6
        out[name] = {"ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2), "gb_s": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "copy_frac": round(gbs / (n * 3 * es / v / 1e6), 4),
                     "plain_ms": round(p, 4), "slowdown": round(ms / p, 3)}
    ctx = {"source": "the paper's Tables 1-2, large arrays, binary64 (Intel Core i5-4200U, AVX2)",
           "paper_one_dotted": {op: round(PAPER_PLAIN_LARGE_F64[op] / v, 3)
                                for op, v in PAPER_ONE_DOTTED_LARGE_F64.items()},
           "paper_both_dotted": {op: round(PAPER_PLAIN_LARGE_F64[op] / v, 3)
                                 for op, v in PAPER_BOTH_DOTTED_LARGE_F64.items()},
           "ours_y_dotted_f64": {op: out["%s_y_dotted_f64" % op]["slowdown"] for op in ("add", "sub", "mul", "div")},
           "ours_both_dotted_f64": dict({op: out["%s_both_dotted_f64" % op]["slowdown"]
                                         for op in ("add", "sub", "mul", "div")},
                                        sqrt=out["sqrt_dotted_f64"]["slowdown"])}
    return {"n": N_STREAM, "forms": out, "paper_context": ctx}


def paper_context(kernels, in_register, cache_resident=None):
    """The paper's slowdowns beside ours (binary64): HBM-resident arrays
    against its large arrays, cache-resident ones against its medium (L3)
    arrays, in-register chains against its L1 arrays.  Context only:
    another machine and another memory system."""
    ops = ("add", "sub", "mul", "div", "sqrt")
    out = {"source": "the paper's Tables 1-2 (Intel Core i5-4200U, AVX2, binary64, twofold operands vs plain)",
           "paper_large_arrays": PAPER_SLOWDOWN_LARGE, "paper_medium_arrays": PAPER_SLOWDOWN_MEDIUM,
           "paper_l1_arrays": PAPER_SLOWDOWN_SMALL,
           "ours_hbm_n2e28": {op: kernels["%s_f64" % op]["slowdown"] for op in ops}}
    if cache_resident:
        out["ours_cache_resident_n2e20"] = {op: cache_resident["ops"]["%s_f64" % op]["slowdown"] for op in ops}
    if in_register:
        out["ours_in_register"] = {op: in_register["ops"]["%s_f64" % op]["twofold"]["slowdown"] for op in ops}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the in-register chains and the batched applications")
    ap.add_argument("--serve-jobs", type=int, default=20000,
                    help="jobs in the serving stream (0 skips it)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 output in DIR and exit")
    ap.add_argument("--profile-command", default="", help="command recorded in the summaries")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.profile_command)
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU only: the twofold hot path runs on a single MI355X here; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1401_6235_amd as tf
    from paper_1401_6235_amd import workloads as W

    tf.lib()  # fail loudly if the HIP library is missing
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    inputs = {}
    for dt in (np.float64, np.float32):
        inputs[np.dtype(dt).name] = make_inputs(torch, dt, W)

    tcalls, pcalls = [], []
    for key, d in inputs.items():
        tag = "f64" if key == "float64" else "f32"
        tcalls += [("%s_%s" % (name, tag), n, fn) for name, n, fn in twofold_calls(tf, d)]
        pcalls += [("%s_%s" % (name, tag), n, fn) for name, n, fn in plain_calls(tf, d)]

    log("timing %d twofold steps (warmup %d)" % (args.steps, args.warmup))
    wall, per = run_pass(torch, tcalls, args.steps, args.warmup)
    log("timing %d plain steps" % args.steps)
    pwall, pper = run_pass(torch, pcalls, args.steps, args.warmup)

    elems = sum(n for _, n, _ in tcalls)
    ms_step = wall / args.steps * 1e3
    value = elems / (wall / args.steps) / 1e9

    kernels = {}
    for name, n, _ in tcalls:
        base, tag = name.rsplit("_", 1)
        es = 8 if tag == "f64" else 4
        words, plain = KERNELS[base]
        p = pper["%s_%s" % (plain, tag)]
        ms = per[name]["ms_avg"]
        kernels[name] = {
            "n": n, "ms": round(ms, 4),
            "gelem_s": round(n / ms / 1e6, 2),
            "gb_s": round(n * words * es / ms / 1e6, 1),
            "hbm_frac": round(n * words * es / ms / 1e6 / HBM_PEAK_GBS, 4),
            "plain_ms": round(p["ms_avg"], 4),
            "plain_gb_s": round(n * PLAIN_WORDS[plain] * es / p["ms_avg"] / 1e6, 1),
            "slowdown": round(ms / p["ms_avg"], 3),
        }
    for tag, es in (("f64", 8), ("f32", 4)):
        v = pper["vmem_" + tag]
        kernels["vmem_" + tag] = {"n": v["n"], "ms": round(v["ms_avg"], 4),
                                  "gb_s": round(v["n"] * 3 * es / v["ms_avg"] / 1e6, 1)}
    for name in list(kernels):  # the HBM rate against the measured copy bandwidth too
        if not name.startswith("vmem"):
            kernels[name]["copy_frac"] = round(kernels[name]["gb_s"] / kernels["vmem_" + name.rsplit("_", 1)[1]]["gb_s"], 4)

    dom = max((k for k in kernels if not k.startswith("vmem")), key=lambda k: kernels[k]["ms"])
    base, tag = dom.rsplit("_", 1)
    es = 8 if tag == "f64" else 4
    alg_bytes = KERNELS[base][0] * es * kernels[dom]["n"]
    achieved = alg_bytes / (kernels[dom]["ms"] * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = traffic_for(dom, src_hash)

    step_bytes = sum(KERNELS[k.rsplit("_", 1)[0]][0] * (8 if k.endswith("f64") else 4) * kernels[k]["n"]
                     for k in kernels if not k.startswith("vmem"))
    plain_ms_step = sum(kernels[k]["plain_ms"] for k in kernels if not k.startswith("vmem"))
    twofold_ms_kernels = sum(kernels[k]["ms"] for k in kernels if not k.startswith("vmem"))

    result = {
        "metric": "twofold Gelem/s, % HBM peak, slowdown vs plain op; serve p50/p99 latency",
        "value": round(value, 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": "twofold hot path, one step = add/sub/mul/div/sqrt/axpy/horner-8 at n=2^28 and "
                        "sum/dot at n=2^26 (ill-conditioned dot instance, cond %.0e), binary64 and binary32"
                        % REDUCE_COND,
            "n_stream": N_STREAM, "n_reduce": N_REDUCE,
            "reduce_cond_achieved": {k: round(v["cond"], 1) for k, v in inputs.items()},
        },
        "hbm_frac_step": round(step_bytes / (twofold_ms_kernels * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "slowdown_step": round(twofold_ms_kernels / plain_ms_step, 3),
        "roofline": {
            "kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "avg_launch_ms": kernels[dom]["ms"],
        },
        "kernels": kernels,
        "kernel_source_hash": src_hash,
    }
    if not args.no_extra:
        log("dotted and mixed operand forms (n = 2^28)")
        result["dotted_forms"] = dotted_forms_run(torch, tf, inputs, pper, args.steps, args.warmup)
    # the timed passes' buffers are no longer needed
    del inputs, tcalls, pcalls
    torch.cuda.empty_cache()
    if not args.no_extra:
        log("in-register chains (n = 2^21, %d steps)" % CHAIN_REPS)
        result["in_register"] = in_register_run(torch, tf, W)
        log("batched applications and fma")
        result["applications"] = applications_run(torch, tf, W)
    if not args.no_extra:
        log("cache-resident elementwise (n = 2^20)")
        result["cache_resident"] = cache_resident_run(torch, tf, W)
    result["paper_context"] = paper_context(kernels, result.get("in_register"), result.get("cache_resident"))
    if args.serve_jobs > 0:
        result["serving"] = serving_run(torch, W, jobs=args.serve_jobs)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)")
        result["cpu_baseline"] = cpu_baseline(W)
        result["cpu_baseline"]["host_cpus"] = os.cpu_count()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
