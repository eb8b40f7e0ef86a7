"""Build the gfx950 HIP library in-tree with hipcc (no JIT cache, no pip install)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", "recon_api.hip")]
OUTPUT = os.path.join(HERE, "librecon.so")
# the same library with the device bounds checks compiled in (recon_debug_violations counts them)
DEBUG_OUTPUT = os.path.join(HERE, "librecon_debug.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # no packed FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # roctx ranges named after the pipeline's stages (shown by rocprofv3 --marker-trace)
         "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def build(verbose=False, output=OUTPUT, extra=()):
    """Compile every HIP source of the library into one shared object (always recompiles)."""
    tmp = output + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    err = "\n".join(l for l in (res.stderr or "").splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, output)
    return output


def build_debug(verbose=False):
    """The library with RECON_DEBUG bounds checks, beside the release one."""
    return build(verbose=verbose, output=DEBUG_OUTPUT, extra=("-DRECON_DEBUG",))


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_debug(verbose=True))
