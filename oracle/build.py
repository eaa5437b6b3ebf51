"""Build the FP64 CPU oracle (test infrastructure) into oracle/libmg_oracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mg_oracle.c")
LIB = os.path.join(HERE, "libmg_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile with gcc, FP contraction off so every rounding is the C source's."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
