"""Serving host logic against a CPU stand-in device (no GPU).

tests/serve_host/fake_device.cpp drives the library's server (admission,
pool, descriptor ring, completion handling from tf_serve_host.hpp) with a
thread in place of the persistent kernel, and prints one JSON line per
scenario.  Built with g++ (host code only): plainly, under ThreadSanitizer,
and under AddressSanitizer with UndefinedBehaviorSanitizer (leak checks
on).
"""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_host", "fake_device.cpp")
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1401_6235_amd", "csrc"),
       "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]


def build(tmp_path, extra=()):
    exe = str(tmp_path / "fake_device")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-pthread", *extra, *INC, "-o", exe, SRC], check=True)
    return exe


def run(exe, env=None):
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    out = {}
    for line in p.stdout.splitlines():
        if line.startswith("{"):
            d = json.loads(line)
            out[d["scenario"]] = d
    return out, p.stderr


def check(res):
    assert res["pool"]["overlap"] == 0 and res["pool"]["accounting"] == 0
    assert res["pool"]["fragments_after_free"] == 1 and res["pool"]["free"] == res["pool"]["cap"]
    assert res["validation"]["fails"] == 0
    for name in ("stream", "tight_budget", "two_slots", "device_restart"):
        r = res[name]
        assert r["completed"] == r["submitted"] == r["unique"], name
        assert r["bad"] == 0 and r["flags_ok"] == 1 and r["fifo"] == 1, name
        assert r["wrong_reject"] == 0, name
        assert r["peak_resident"] <= r["budget"], name
    assert res["tight_budget"]["waits"] > 0          # the budget forced the queue head to wait
    assert res["two_slots"]["max_in_flight"] <= 2     # slots bound the jobs in flight
    assert res["stream"]["max_in_flight"] > 8         # continuous batching: many jobs at once
    # a drained worker is relaunched by the next publish, and not before:
    # with nothing in flight it stays down through the 200 ms pause (ten
    # idle periods; relaunching on every drain would start it ~10 times),
    # so other work can use its hardware queue
    assert 2 <= res["device_restart"]["starts"] <= 3


def test_server_host_logic(tmp_path):
    res, _ = run(build(tmp_path))
    check(res)


def test_server_host_logic_under_thread_sanitizer(tmp_path):
    exe = build(tmp_path, ["-fsanitize=thread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    res, err = run(exe, env)
    assert "ThreadSanitizer" not in err, err[:4000]
    check(res)


def test_server_host_logic_under_address_and_undefined_sanitizers(tmp_path):
    exe = build(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"])
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1:exitcode=66",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=67")
    res, err = run(exe, env)
    assert "AddressSanitizer" not in err and "runtime error" not in err and "LeakSanitizer" not in err, err[:4000]
    check(res)
