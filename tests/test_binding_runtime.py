"""The binding loads torch before the HIP library, so the process has one
HIP runtime: the library binds to the copy torch loaded instead of a second
one from the system path, which would not know torch's device memory (every
launch on a torch tensor would then fail).  Checked in a fresh process on
the CPU: after lib(), exactly one libamdhip64 is mapped."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import paper_1401_6235_amd as tf
tf.lib()
maps = open('/proc/self/maps').read()
print(sorted(set(l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l)))
"""


def test_one_hip_runtime_after_loading_the_library():
    p = subprocess.run([sys.executable, "-c", CODE], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stderr[-3000:]
    runtimes = ast.literal_eval(p.stdout.strip().splitlines()[-1])
    assert len(runtimes) == 1, runtimes
