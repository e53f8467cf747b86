"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C compiled by gcc with OpenMP over the batch and with
floating-point contraction disabled, so that its float variant does plain
float multiplies and adds.  It shares no source with the GPU library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kron_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile kron_oracle.c into oracle/liboracle.so and return its path."""
    return build_to(LIB, extra_flags=extra_flags, verbose=verbose)


def build_to(out_path: str, extra_flags=(), verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", *extra_flags, SRC, "-o", out_path]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
