"""Build the CPU oracle (plain C) into oracle/liboracle.so.

Test infrastructure: the oracle is compiled with -O2 -ffp-contract=off and no
fast-math so that its single-precision UCT arithmetic rounds once per
operation, in the stated order.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["rules.c", "mcts.c", "valuenet.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src_dir: str = HERE, out: str = LIB) -> str:
    """Compile the sources of `src_dir` (default: this folder) into `out`."""
    srcs = [os.path.join(src_dir, s) for s in SOURCES if os.path.exists(os.path.join(src_dir, s))]
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-mfpmath=sse",
           "-msse2", "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", out + ".tmp"] + srcs + ["-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
