"""Build the C++ consumer of the C ABI (tests/c_abi/abi_check.bin): host code
only, linked against the library and the test oracle with run paths to
their directories."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "abi_check.cpp")
BIN = os.path.join(HERE, "abi_check.bin")


def build() -> str:
    pkg, orc = os.path.join(ROOT, "paper_1401_6235_amd"), os.path.join(ROOT, "oracle")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           SRC, "-o", BIN + ".tmp", "-L", pkg, "-ltwofold", "-L", orc, "-ltforacle",
           "-Wl,-rpath,$ORIGIN/../../paper_1401_6235_amd", "-Wl,-rpath,$ORIGIN/../../oracle"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build())
