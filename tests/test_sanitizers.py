"""The host C code under AddressSanitizer and UndefinedBehaviorSanitizer (no
GPU).

The oracle (oracle/tf_oracle.c) and the exact ill-conditioned-dot generator
(paper_1401_6235_amd/workloads/illdot.c) are rebuilt with
-fsanitize=address,undefined and every oracle, generator and workload test
is run again against those builds in a child process, the sanitizer runtime
preloaded and every report fatal.  A planted out-of-bounds read (a call
with n past the end of its arrays) shows that the instrumentation is live.
The serving host logic has its own sanitizer runs in test_serve_host.py.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ORACLE_TESTS = ["test_oracle_eft.py", "test_oracle_bounds.py", "test_oracle_paper.py", "test_oracle_tree.py",
                "test_oracle_coupled.py", "test_oracle_apps.py", "test_workloads.py"]


def _asan_runtime():
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()


def _build(tmp_path):
    orc = str(tmp_path / "libtforacle_san.so")
    gen = str(tmp_path / "libtfgen_san.so")
    subprocess.run(["gcc", *SAN, "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", orc, os.path.join(ROOT, "oracle", "tf_oracle.c"), "-lm"], check=True)
    subprocess.run(["gcc", *SAN, "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", gen,
                    os.path.join(ROOT, "paper_1401_6235_amd", "workloads", "illdot.c"), "-lm"], check=True)
    return orc, gen


def _env(orc, gen):
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = _asan_runtime() + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=66"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=67"
    env["TF_ORACLE_LIB"] = orc
    env["TF_WORKLOADS_LIB"] = gen
    return env


def test_oracle_and_generator_tests_pass_under_sanitizers(tmp_path):
    orc, gen = _build(tmp_path)
    env = _env(orc, gen)
    # the child really loads the instrumented builds
    probe = ("import oracle; from paper_1401_6235_amd import workloads as W; "
             "assert oracle.lib()._name == %r, oracle.lib()._name; W.illdot_case(64, 1e8, seed=3); "
             "assert W._gen_lib()._name == %r, W._gen_lib()._name; "
             "maps = open('/proc/self/maps').read(); assert 'libasan' in maps and 'libubsan' in maps" % (orc, gen))
    p = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 0, p.stdout + p.stderr
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", t) for t in ORACLE_TESTS]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-6000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-6000:]
    assert " passed" in p.stdout


def test_planted_overflow_is_reported(tmp_path):
    """Negative control: the oracle's plain add asked for 100 elements of
    arrays that hold 10 reads past their end, which the instrumented build
    must report."""
    orc, gen = _build(tmp_path)
    env = _env(orc, gen)
    code = ("import ctypes as C, numpy as np, oracle; x = np.ones(10); z = np.zeros(100); "
            "f = oracle.lib().orc_plain_add_f64; "
            "f(C.c_int64(100), C.c_void_p(x.ctypes.data), C.c_void_p(x.ctypes.data), C.c_void_p(z.ctypes.data))")
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert p.returncode != 0
    assert "heap-buffer-overflow" in p.stderr, p.stderr[-3000:]
