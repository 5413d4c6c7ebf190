"""Compiles the CPU oracle (test infrastructure only) into oracle/libppp_oracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ppp_oracle.c")
LIB = os.path.join(HERE, "libppp_oracle.so")


def build(force: bool = True) -> str:
    """Builds the oracle with gcc.  -ffp-contract=off keeps every product and
    sum separately rounded, so the oracle's arithmetic is the one written."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
