"""Build the CPU oracle (test infrastructure only) into oracle/libblp_oracle.so.

Plain gcc, FP64, -O2 -ffp-contract=off (no fused multiply-add contraction),
no fast-math, so the oracle rounds every operation as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "blp_oracle.c")
LIB = os.path.join(HERE, "libblp_oracle.so")


def build_oracle(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle())
