"""Compile the FP64 CPU oracle into ``oracle/libbtrirt_oracle.so``.

Test infrastructure only.  ``-ffp-contract=off`` keeps every product and sum
rounded as written; OpenMP splits only the per-row loops (no reductions run in
parallel), so results do not depend on the thread count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "btrirt_oracle.c")
LIB = os.path.join(HERE, "libbtrirt_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_native(dest_dir: str, verbose: bool = False) -> str:
    """The same source built at -O3 for the host's own instruction set, into
    dest_dir (for timing the oracle on the machine that runs it; a binary
    built for one CPU is never shipped to another)."""
    out = os.path.join(dest_dir, "libbtrirt_oracle_native.so")
    flags = [f for f in CFLAGS if f != "-O2"] + ["-O3", "-march=native"]
    cmd = ["gcc", *flags, SRC, "-o", out, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
