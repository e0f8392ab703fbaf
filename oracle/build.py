"""Compile the C oracle into oracle/liboracle.so (plain gcc, -O2, no SIMD intrinsics).

Test infrastructure: the product library never builds or loads this."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# A test may point the loader at a deliberately broken copy of the oracle.
LOAD_PATH = os.environ.get("RVE_ORACLE_LIB") or LIB


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, SRC, "-lm", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True), file=sys.stderr)
