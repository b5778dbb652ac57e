"""Build the gfx950 HIP library libdvc.so in place (next to this file), and
the measurement library measure/libvalu_probe.so.

hipcc --offload-arch=gfx950, one translation unit (csrc/dvc_lib.hip),
-ffp-contract=off so that single-precision UCT arithmetic rounds once per
operation, correctly rounded division and square root (the hipcc default),
and packed-FP32 instructions disabled.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "dvc_lib.hip")
LIB = os.path.join(HERE, "libdvc.so")
PROBE_SRC = os.path.join(HERE, "measure", "valu_probe.hip")
PROBE_LIB = os.path.join(HERE, "measure", "libvalu_probe.so")


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def flags(arch: str = "gfx950"):
    return ["--offload-arch=" + arch, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def _compile(src: str, out: str, verbose: bool, extra=()):
    cmd = [hipcc()] + flags() + list(extra) + ["-o", out + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False, extra=()) -> str:
    _compile(SRC, LIB, verbose, extra)
    _compile(PROBE_SRC, PROBE_LIB, verbose, extra)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=[a for a in sys.argv[1:] if a.startswith("-")])
