#!/usr/bin/env python3
"""Benchmark of the twofold hot path on one MI355X.

One step = one pass of every twofold kernel of the hot path over resident
synthetic inputs, binary64 and binary32:
    add, sub, mul, div, sqrt   (both operands twofold)   n = 2^28
    axpy  (a = (0.7, 1e-17))                             n = 2^28
    Horner, degree 8                                     n = 2^28
    sum (twofold leaves), dot (plain vectors)            n = 2^26, cond 1e16
The same pass with the plain (non-twofold) kernels and the memory probe is
timed right after, for the twofold/plain slowdown.  value = twofold
elements per second over the step (input elements for the reductions).

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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1401_6235_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, name), "rb").read())
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
    """The oracle (single-threaded scalar C) on a bounded sample of the
    step: every kernel of the step on n = 2^20 elements (2^20 leaves for
    the reductions), binary64 and binary32."""
    import numpy as np
    import oracle
    n = 1 << 20
    total_elems = 0
    t_total = 0.0
    for dt in (np.float64, np.float32):
        c = W.elementwise("add", n, seed=0, dtype=dt)
        s = W.elementwise("sqrt", n, seed=0, dtype=dt)
        h = W.horner_case(n, seed=0, dtype=dt)
        r = W.illdot_case(n, REDUCE_COND, seed=0, dtype=dt)
        hi, lo = W.product_split(r["x"], r["y"])
        a = W.axpy_case(1, dtype=dt)["a"]
        jobs = [
            lambda: oracle.add(c["x0"], c["x1"], c["y0"], c["y1"]),
            lambda: oracle.sub(c["x0"], c["x1"], c["y0"], c["y1"]),
            lambda: oracle.mul(c["x0"], c["x1"], c["y0"], c["y1"]),
            lambda: oracle.div(c["x0"], c["x1"], c["y0"], c["y1"]),
            lambda: oracle.sqrt(s["x0"], s["x1"]),
            lambda: oracle.axpy(a, c["x0"], c["x1"], c["y0"], c["y1"]),
            lambda: oracle.horner(h["c"], h["x0"], h["x1"]),
            lambda: oracle.sum(hi, lo),
            lambda: oracle.dot(r["x"], None, r["y"], None),
        ]
        reps = 0
        t0 = time.perf_counter()
        while True:
            for j in jobs:
                j()
            reps += 1
            if time.perf_counter() - t0 > seconds_target / 2:
                break
        t_total += time.perf_counter() - t0
        total_elems += reps * n * len(jobs)
    return {"value": total_elems / t_total / 1e9, "unit": "Gelem/s", "cores": 1, "kind": "oracle",
            "sample": "every kernel of the step (add, sub, mul, div, sqrt, axpy, horner-8, sum, dot), "
                      "binary64 and binary32, on n = 2^20 elements each, single thread, %.1f s" % t_total}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
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
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)")
        result["cpu_baseline"] = cpu_baseline(W)
        result["cpu_baseline"]["host_cpus"] = os.cpu_count()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
