"""Host logic of the library under AddressSanitizer / UBSan, on the CPU.

The library's sources are built with the host code instrumented and linked against a mock of
the HIP runtime (tests/hostmock/mock_hip.cpp: host memory, kernels that do nothing, streams /
events / graphs whose use after destruction the sanitizer reports, and CUDA's capture rules).
The driver (tests/hostmock/driver.cpp) makes the batched tests' calls with their shapes,
including the 512-pool workload, and checks the host bookkeeping: a batched call captures one
graph for new arguments or a replaced handle and replays it otherwise; a released handle's
workspace serves the next handle without a new allocation; the allocation-free entry point
allocates and frees nothing.  A second run reports every batched pool as overflowing, so that
each takes the single-pool path.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2501_07642_amd import inputs  # noqa: E402

HOSTMOCK = os.path.join(ROOT, "tests", "hostmock")


@pytest.fixture(scope="module")
def driver():
    sys.path.insert(0, HOSTMOCK)
    import build_hostmock

    path = build_hostmock.DRIVER
    sources = [os.path.join(HOSTMOCK, f) for f in ("mock_hip.cpp", "driver.cpp")]
    from paper_2501_07642_amd import build as lib
    sources += [os.path.join(lib.CSRC, f) for f in os.listdir(lib.CSRC)]
    if not os.path.exists(path) or os.path.getmtime(path) < max(os.path.getmtime(s) for s in sources):
        build_hostmock.build()
    return path


@pytest.fixture(scope="module")
def shapes_file(tmp_path_factory):
    w = inputs.WORKLOADS["batched_512"]
    path = tmp_path_factory.mktemp("hostmock") / "shapes.txt"
    path.write_text("".join(f"{n} {n1} {d}\n" for n, n1, d in inputs.batched_shapes(w["num_problems"], w["shape_seed"])))
    return str(path)


def run(driver, shapes_file, flags_set):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.pop("RR_TUNE_FILE", None)
    if flags_set:
        env["RR_MOCK_FLAGS_SET"] = "1"
    else:
        env.pop("RR_MOCK_FLAGS_SET", None)
    r = subprocess.run([driver, shapes_file], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ALL OK" in r.stdout, out[-6000:]
    return r.stdout


def test_host_logic_under_sanitizers(driver, shapes_file):
    out = run(driver, shapes_file, flags_set=False)
    for name in ("graph captured once, replayed for the same arguments",
                 "replaced handle with the same arguments: a new graph",
                 "the next handle's first call reuses the released workspace",
                 "allocation-free entry point allocates and frees nothing",
                 "after the first stream is destroyed: a third stream, the second, the null stream",
                 "the 512-pool workload"):
        assert f"CHECK {name} ok" in out


def test_host_logic_single_pool_fallback(driver, shapes_file):
    out = run(driver, shapes_file, flags_set=True)
    assert "CHECK the 512-pool workload ok" in out
