"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, no GPU toolchain.  `python oracle/build_oracle.py` or
`build_oracle.build()`.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


FLAGS = ["-std=c11", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
         "-Wall", "-Wextra"]


def build(verbose=False, native=False, dst=None):
    """Compile md_oracle.c into dst (default oracle/liboracle.so).  native
    adds -march=native: code for the CPU that compiles it, so such a build is
    only loaded on the host that made it (the CPU baseline of bench.py)."""
    src = os.path.join(HERE, "md_oracle.c")
    out = dst or LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + FLAGS + (["-march=native"] if native else []) + ["-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
