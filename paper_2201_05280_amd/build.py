"""Build the HIP library for gfx950 in-tree (hipcc, no torch extension)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpgk.so")
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("pgk.hip", "batch.hip", "mlp.hip")]
PROBE_LIB = os.path.join(HERE, "libpgk_probe.so")
PROBE_SOURCES = [os.path.join(HERE, "csrc", "probe.hip")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    # no packed FP32 instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _hipcc(out, sources, extra=(), verbose=True):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + HIPCC_FLAGS + list(extra) + ["-I", os.path.join(ROOT, "include"),
                                                 "-I", os.path.join(HERE, "csrc"),
                                                 "-o", out + ".tmp"] + sources
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)


def build(verbose=True, extra=()):
    """libpgk.so (the method) and libpgk_probe.so (bandwidth reference copies)."""
    _hipcc(LIB, SOURCES, extra, verbose)
    _hipcc(PROBE_LIB, PROBE_SOURCES, extra, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
