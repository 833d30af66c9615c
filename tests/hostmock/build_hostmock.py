"""Build the host-logic test driver: librr's sources with the host code under AddressSanitizer
and UBSan, linked against the mock runtime in this directory instead of the HIP runtime.

Usage: python tests/hostmock/build_hostmock.py   (or build() from Python); writes
_build/hostmock/rr_hostmock_driver.  Every call recompiles.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(ROOT, "_build", "hostmock")
DRIVER = os.path.join(OUT, "rr_hostmock_driver")
sys.path.insert(0, ROOT)


def build(verbose=False):
    from paper_2501_07642_amd import build as lib

    os.makedirs(OUT, exist_ok=True)
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={lib.ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Wno-unused-result",
             "-I", os.path.join(ROOT, "include")]
    sources = [os.path.join(lib.CSRC, s) for s in lib.SOURCES]
    sources += [os.path.join(HERE, "mock_hip.cpp"), os.path.join(HERE, "driver.cpp")]

    def compile_one(src):
        obj = os.path.join(OUT, os.path.splitext(os.path.basename(src))[0] + ".o")
        r = subprocess.run([lib.hipcc(), *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, sources))
    clang = os.path.join(os.path.dirname(os.path.realpath(lib.hipcc())), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = shutil.which("amdclang++") or "/opt/rocm/llvm/bin/clang++"
    # linked without the HIP runtime: the mock defines every runtime entry the objects use
    r = subprocess.run([clang, "-fsanitize=address,undefined", "-o", DRIVER, *objs, "-lstdc++"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    if verbose:
        print("built", DRIVER)
    return DRIVER


if __name__ == "__main__":
    build(verbose=True)
