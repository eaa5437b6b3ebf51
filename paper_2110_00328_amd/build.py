"""Build the HIP library libmggpu.so for gfx950 (in-tree)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "mggpu.hip")
# host-only sources linked into the same library
HOST_SRC = [os.path.join(HERE, "csrc", "mg_background.cpp")]
LIB = os.path.join(HERE, "libmggpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           # no packed FP32 instructions (v_pk_*_f32) in any HIP code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-Wall", "-Wno-unused-function", "-o", LIB + ".tmp", SRC] + HOST_SRC
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
