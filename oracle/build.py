"""Build the FP64 oracle (plain C + OpenMP) into oracle/libbbref.so.

Test infrastructure: compiled so the checker exists, never linked into the
HIP library.  No fast-math: the oracle relies on IEEE 1/0 = inf and NaN
propagation.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "libbbref.so")
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", out + ".tmp", os.path.join(HERE, "bbref.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
