"""Builds tests/probe/libmfma_probe.so (gfx950), the MFMA rounding probe the GPU tests load."""

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmfma_probe.so")


def build(verbose=False):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    arch = os.environ.get("RR_OFFLOAD_ARCH", "gfx950")
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={arch}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(HERE, "mfma_probe.hip"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for the MFMA probe:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
