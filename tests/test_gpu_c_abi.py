"""GPU: a C++ program that uses only tf.h, hipMalloc and raw pointers
(tests/c_abi/abi_check.cpp) calls the library and checks the results bit
for bit against the oracle, plus the error codes of misuse."""
import os
import subprocess

import pytest

from gpu_util import step, torch_cuda

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "abi_check.bin")


def test_c_consumer_matches_oracle():
    torch_cuda()
    assert os.path.exists(BIN), "abi_check.bin missing: run __graft_entry__.build()"
    step("C ABI consumer")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout
