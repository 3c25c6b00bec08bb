"""Host code of the library under AddressSanitizer / UndefinedBehaviorSanitizer.

The C++ sources of the planner, executor, batch issue and C ABI are
built with g++ against a host-only stand-in for the HIP runtime
(tests/hostsim/hip_stub.cpp) and driven through every host path the GPU
tests take (tests/hostsim/driver.cpp).  The stand-in checks every stage-kernel
launch's tile address range against its allocations (every tile of a
grouped launch's device table included), the thread and LDS limits, and the stream / event / graph-capture rules (fork-join closure,
no synchronisation inside a capture, no use of destroyed handles).  Any
sanitizer report, flagged launch, failed expectation or leaked allocation
fails the test.
"""
import os
import shutil
import subprocess

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_12209_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "hostsim")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("hostsim") / "driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-Wno-unused-result", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-o", exe,
           os.path.join(HERE, "driver.cpp"), os.path.join(HERE, "hip_stub.cpp"),
           os.path.join(CSRC, "runtime.cpp"), os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "batch.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


def _run(exe, args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=600)


def test_host_paths_clean_under_sanitizers(driver):
    shapes = synth.batch_sizes()
    args = [str(len(shapes))] + [str(v) for (nz, ny, nx) in shapes for v in (nx, ny, nz)]
    res = _run(driver, args)
    assert res.returncode == 0 and "hostsim ok" in res.stdout, (res.stdout[-2000:], res.stderr[-6000:])
