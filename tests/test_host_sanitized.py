"""The C ABI's host logic under AddressSanitizer and UndefinedBehaviorSanitizer
on the CPU: ga_api.hip built with g++ against a host-only stand-in for the HIP
runtime (tests/host_mock: device memory is host memory, kernels are stubs that
check the tables and launch shapes handed to them, a graph destroyed while in
flight aborts), driven by tests/host_mock/replay.py through the Python
binding in a child interpreter with the sanitizer runtimes preloaded: single
runs in every form, schedule and genome variant, resume, argument errors, the
64-run batch with launch-shape changes and membership churn, the served
stream through the run pool, the relatedness calls. Any report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MOCK = os.path.join(ROOT, "tests", "host_mock")


def _runtime(name: str) -> str:
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not found")
    return path


def test_host_logic_under_sanitizers(tmp_path):
    so = str(tmp_path / "libga_host_mock.so")
    build = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fPIC", "-shared",
             "-I" + MOCK, "-I" + os.path.join(ROOT, "paper_2405_03605_amd", "csrc"),
             "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
             "-x", "c++", os.path.join(ROOT, "paper_2405_03605_amd", "csrc", "ga_api.hip"),
             "-x", "c++", os.path.join(MOCK, "mock_hip.cpp"), "-o", so]
    subprocess.run(build, check=True, capture_output=True, timeout=600)
    env = dict(os.environ,
               LD_PRELOAD=f"{_runtime('libasan.so')}:{_runtime('libubsan.so')}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(MOCK, "replay.py"), so], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    tail = r.stdout[-3000:] + "\n" + r.stderr[-5000:]
    assert r.returncode == 0, tail
    for line in ("single runs ok", "batched ok", "served ok 300", "relatedness ok"):
        assert line in r.stdout, tail
