"""Build the UMI HIP library (libumi.so) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libumi.so")
SOURCES = ["umi_kernels.hip", "umi_host.hip", "umi_server.hip"]
DIAG_PATH = os.path.join(HERE, "libumi_diag.so")   # measurement aid (FMA throughput)
DIAG_SOURCES = ["umi_diag.hip"]
ARCH = "gfx950"

# Packed FP32 VALU forms are switched off for every device compilation.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build_library(out: str = LIB_PATH, extra: list[str] | None = None, verbose: bool = False,
                  sources: list[str] | None = None) -> str:
    """Compile every HIP source of the library into one shared object."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-result", *DEVICE_FLAGS, "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(CSRC, s) for s in (sources or SOURCES)], "-o", tmp]
    if extra:
        cmd[1:1] = extra
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_all(verbose: bool = False):
    """The library and the measurement aid."""
    return [build_library(LIB_PATH, verbose=verbose),
            build_library(DIAG_PATH, verbose=verbose, sources=DIAG_SOURCES)]


if __name__ == "__main__":
    print("\n".join(build_all(verbose="-v" in sys.argv)))
