"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use the
oracle.  It is compiled with gcc, strict IEEE semantics (no fast-math, no
floating-point contraction) and OpenMP.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "euler_oracle.c")
LIBRARY = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
          "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(source=SOURCE, output=LIBRARY, extra_flags=(), quiet=True):
    """Compile `source` into the shared library `output`; return its path."""
    cmd = ["gcc", *CFLAGS, *extra_flags, source, "-o", output + ".tmp", "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    if res.stderr and not quiet:
        sys.stderr.write(res.stderr)
    os.replace(output + ".tmp", output)
    return output


if __name__ == "__main__":
    print(build(quiet=False))
