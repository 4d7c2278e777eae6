"""The library's host code on the CPU against a stand-in of the HIP runtime.

Every source is compiled host-only with AddressSanitizer and
UndefinedBehaviorSanitizer and linked with tests/host_mock/mock_hip.cpp
(streams, events, graph capture and launch modelled; kernels checked, not
run).  The entry-point driver of tests/host_asan then runs every host path:
plans, workspace growth, graph capture, cache, replay and eviction, the fork
and join of the second stream, batches, the asynchronous and no-allocation
entry points, warm starts, the data form, the autotuner and the error paths.
The stand-in also checks the rules of stream capture the library relies on
(no synchronisation, copy or allocation while capturing; every forked stream
joined back; no use of destroyed objects); a self-test shows that each rule
check fires."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "mock")


@pytest.fixture(scope="module")
def built():
    if not (os.path.exists("/opt/rocm/bin/hipcc") and os.path.exists("/opt/rocm/llvm/bin/clang++")):
        pytest.skip("no ROCm compiler")
    r = subprocess.run(["bash", "tests/host_mock/build.sh"], cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    return OUT


def _run(path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([path], capture_output=True, text=True, timeout=600, env=env)


def test_stand_in_rule_checks(built):
    r = _run(os.path.join(built, "selftest"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "stand-in self-test: 0 failed" in r.stdout


def test_host_paths_under_sanitizers(built):
    r = _run(os.path.join(built, "driver"))
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "0 rule violations" in out and "host sanitizer run: 0 failed checks" in out, out[-4000:]
