"""Host logic of the benchmark (no GPU): the map from kernel names to bench
keys against the names rocprofv3 recorded in the committed profiles, the
algorithmic bytes per launch, and the profile summarizer run on a miniature
rocprofv3 output (scale factors calibrated on the copy kernel, traffic per
launch, and only the benchmark's own grid kept for each kernel)."""
import csv
import glob
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_keys_of_the_profiled_kernel_names():
    seen = 0
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_kernel_trace.txt")):
        for line in open(path):
            if line.startswith("#") or line.startswith("bench_key"):
                continue
            key, _calls, _avg, _grid, name = line.rstrip("\n").split(None, 4)
            assert bench.bench_key(name) == key, (path, name)
            seen += 1
    assert seen >= 30
    # kernels outside the benchmark's set map to nothing
    assert bench.bench_key("void tf::reduce_last_kernel<double, false>(long, long)") is None
    assert bench.bench_key("void tf::ew_vec_kernel<double, 0, false, true, 1>(long)") is None
    assert bench.bench_key("__amd_rocclr_fillBufferAligned") is None


def test_algorithmic_bytes_per_launch():
    n, r = bench.N_STREAM, bench.N_REDUCE
    assert bench.alg_bytes("add_f64") == 6 * 8 * n      # x0 x1 y0 y1 in, z0 z1 out
    assert bench.alg_bytes("sqrt_f32") == 4 * 4 * n
    assert bench.alg_bytes("horner_f64") == 4 * 8 * n
    assert bench.alg_bytes("sum_f64") == 2 * 8 * r      # twofold leaves, nothing written per leaf
    assert bench.alg_bytes("dot_f32") == 2 * 4 * r      # dotted x and y
    assert bench.alg_bytes("vmem_f64") == 3 * 8 * n
    assert bench.alg_bytes("plain_add_f64") == 3 * 8 * n
    assert bench.alg_bytes("plain_sum_f32") == 1 * 4 * r
    m, ns = bench.JORDAN_M, bench.JORDAN_NSYS
    assert bench.alg_bytes("jordan3_f64") == (m * (m + 1) + 4 * m) * 8 * ns
    assert bench.alg_bytes("plain_jordan3_f64") == (m * (m + 1) // 2 + 2 * m) * 8 * ns
    assert bench.alg_bytes("fma_f32") == 8 * 4 * bench.FMA_N
    assert bench.alg_bytes("unknown_f64") is None


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


VMEM64 = "void tf::plain_vec_kernel<double, 99, 4>(long, double const*, double const*, double*)"
VMEM32 = "void tf::plain_vec_kernel<float, 99, 4>(long, float const*, float const*, float*)"
ADD64 = "void tf::ew_vec_kernel<double, 0, true, true, 1>(long, double const*, double const*, double const*)"
SUM32 = "void tf::reduce_tiles_kernel<float, 1, 8, true>(long, long, int, int, float const*, float const*)"


def test_summarizer_on_a_miniature_profile(tmp_path):
    n, r = bench.N_STREAM, bench.N_REDUCE
    big = {VMEM64: n // 8, VMEM32: n // 16, ADD64: n // 2, SUM32: r // 16}  # grid sizes
    trace = []
    for name, grid, ns in ((VMEM64, big[VMEM64], 1000), (VMEM64, big[VMEM64], 1200), (VMEM64, 4096, 5),
                           (VMEM32, big[VMEM32], 600), (ADD64, big[ADD64], 2000), (ADD64, 1024, 3),
                           (SUM32, big[SUM32], 80)):
        t0 = 10 ** 9 + len(trace) * 10 ** 6
        trace.append({"Kernel_Name": name, "Grid_Size_X": grid, "Start_Timestamp": t0,
                      "End_Timestamp": t0 + ns})
    _write_csv(str(tmp_path / "prof" / "trace" / "x_kernel_trace.csv"), trace)
    # FETCH_SIZE reads half of the bytes read and WRITE_SIZE the bytes
    # written, in KiB; the small-grid dispatches carry nonsense that must
    # not be used
    read = {VMEM64: 2 * 8 * n, VMEM32: 2 * 4 * n, ADD64: 4 * 8 * n, SUM32: 2 * 4 * r}
    wrote = {VMEM64: 8 * n, VMEM32: 4 * n, ADD64: 2 * 8 * n, SUM32: 0}
    for which, val in (("fetch", lambda k: read[k] / 2 / 1024), ("write", lambda k: wrote[k] / 1024)):
        rows = [{"Kernel_Name": k, "Grid_Size": big[k], "Counter_Name": which.upper() + "_SIZE",
                 "Counter_Value": val(k)} for k in big]
        rows += [{"Kernel_Name": ADD64, "Grid_Size": 1024, "Counter_Name": which.upper() + "_SIZE",
                  "Counter_Value": 1e12}]
        _write_csv(str(tmp_path / "prof" / which / "x_counter_collection.csv"), rows)
    out = tmp_path / "out"
    bench.summarize_profiles(str(tmp_path / "prof"), "the command", out_dir=str(out))
    t = json.load(open(out / "traffic.json"))
    assert t["source_hash"] == bench.kernel_source_hash()
    assert t["scale"] == {"f64": {"fetch": 2.0, "write": 1.0}, "f32": {"fetch": 2.0, "write": 1.0}}
    assert t["kernels"]["add_f64"]["bytes_per_launch"] == 6 * 8 * n
    assert t["kernels"]["add_f64"]["algorithmic_bytes"] == 6 * 8 * n
    assert t["kernels"]["sum_f32"]["bytes_per_launch"] == 2 * 4 * r
    lines = open(out / "hot_path_step_n2e28_kernel_trace.txt").read().splitlines()
    assert "# command: the command" in lines
    row = {l.split()[0]: l.split() for l in lines if not l.startswith("#")}
    assert row["vmem_f64"][1:3] == ["2", "1.10"]   # the two large-grid launches only, 1.1 us average
    assert row["add_f64"][1:4] == ["1", "2.00", str(big[ADD64])]
    ratios = [l.split()[-1] for l in open(out / "hot_path_step_n2e28_counters.txt") if l.startswith(("add_", "sum_"))]
    assert ratios == ["1.0000", "1.0000"]


def test_source_hash_ignores_comments_only():
    src = ('int a = 1; // note\nconst char *s = "x // kept /* kept */"; /* block\n comment */ char q = \'/\';\n'
           "char e = '\\''; // end")
    out = bench.strip_comments(src)
    assert "note" not in out and "block" not in out and "end" not in out
    assert '"x // kept /* kept */"' in out and "'/'" in out and "'\\''" in out
    assert bench.strip_comments("a = b / c; // x") == "a = b / c;  "
    # a comment edit keeps the hash, a code edit changes it
    assert bench.strip_comments("x = 1; // one") == bench.strip_comments("x = 1; // two")
    assert bench.strip_comments("x = 1;") != bench.strip_comments("x = 2;")


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
