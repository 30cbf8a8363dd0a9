"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is plain C compiled by gcc with floating-point contraction off so
that every binary64 operation is evaluated as written, and with OpenMP for
its loops over protozoa (one thread unless oracle_set_threads asks for
more; results do not depend on the thread count)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "apo_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fvisibility=hidden", "-fopenmp", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
