"""Build the CPU oracle (test infrastructure only) into oracle/libblp_oracle.so.

Plain gcc, FP64, -O2 -ffp-contract=off (no fused multiply-add contraction),
no fast-math, so the oracle rounds every operation as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "blp_oracle.c"), os.path.join(HERE, "blp_oracle_1d.c")]
HDR = os.path.join(HERE, "blp_oracle.h")
LIB = os.path.join(HERE, "libblp_oracle.so")


def build_oracle(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(f) for f in SRCS + [HDR]):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", tmp] + SRCS + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle())
