"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer: the
same C source built with both (any report aborts the process), loaded in a
child interpreter with the sanitizer runtimes preloaded, running every oracle
pin (determinism and resume included) and the host phylogeny checks. CPU only."""
import glob
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.basename(__file__)

PINS = sorted(os.path.relpath(p, ROOT)
              for p in glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py"))
              if os.path.basename(p) != HERE) + ["tests/test_phylo_cpu.py"]


def _runtime(name: str) -> str:
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not found")
    return path


def test_oracle_pins_under_sanitizers(tmp_path):
    so = oracle.build_sanitized(tmp_path / "libga_oracle_san.so")
    env = dict(os.environ,
               GA_ORACLE_LIB=so,
               LD_PRELOAD=f"{_runtime('libasan.so')}:{_runtime('libubsan.so')}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + PINS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-4000:] + "\n" + r.stderr[-4000:])
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "error" not in r.stdout.lower().split("passed")[-1], tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
