"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so.

gcc, -ffp-contract=off so that no multiply-add is fused behind the source's
back (every fused multiply-add in the oracle is an explicit fma() call),
OpenMP over output columns.  -mfma -mavx2 make fma() a single instruction on
any x86-64-v3 host; the arithmetic is the same either way.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["dd_oracle.c", "ozaki_oracle.c", "cdd_oracle.c", "potrf_oracle.c", "qd_oracle.c"]
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-mfma", "-mavx2", "-Wall", "-Wno-unknown-pragmas"]


def build(out=LIB, sources=None, extra=(), cwd=HERE, quiet=True):
    """Compile the oracle sources (relative to cwd) into `out`."""
    srcs = sources if sources is not None else [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", *CFLAGS, *extra, "-I", HERE, *srcs, "-o", out, "-lm"]
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + " ".join(cmd) + "\n" + r.stderr)
    if not quiet and r.stderr:
        sys.stderr.write(r.stderr)
    return out


if __name__ == "__main__":
    print(build(quiet=False))
