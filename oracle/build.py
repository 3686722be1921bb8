"""Build the FP64 CPU oracle (test infrastructure) into ``oracle/libcuesim_oracle.so``.

Plain gcc, -O2, OpenMP over rows/cones, no fast-math: the oracle's arithmetic must stay
IEEE FP64 exactly as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "cuesim_oracle.c")
LIBRARY = os.path.join(HERE, "libcuesim_oracle.so")


def build(source=SOURCE, output=LIBRARY, extra_flags=(), verbose=False):
    """Compile ``source`` into the shared library ``output``; returns its path."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", "-Wextra", "-I", HERE, *extra_flags,
           source, "-o", output + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(output + ".tmp", output)
    return output


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
