"""Pins for the oracle's Philox4x32-10 (the RNG named for the counter-based
contract): the published known-answer vectors, and an independent library
implementation (rocRAND's open-source engine compiled for the host)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(x, 16) for x in line.split()])
    return rows


def test_known_answer_vectors():
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        out = oracle.philox(r[0:4], r[4:6])
        assert [int(x) for x in out] == r[6:10]


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    exe = tmp_path_factory.mktemp("rr") / "rocrand_philox_ref"
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(GOLDEN, "rocrand_philox_ref.cpp"), "-o", str(exe)],
                   check=True)
    return str(exe)


def test_against_rocrand_engine(rocrand_ref):
    rng = np.random.default_rng(20240503)
    inputs = rng.integers(0, 2**32, size=(4000, 6), dtype=np.uint64)
    # include counters shaped like the GA's (slot, island, generation, tag)
    inputs[:8, 0] = np.arange(8)
    inputs[:8, 3] = np.arange(8) % 3
    text = "\n".join(" ".join(f"{int(v):08x}" for v in row) for row in inputs) + "\n"
    res = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(x, 16) for x in ln.split()] for ln in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    assert ref.shape == (4000, 4)
    ours = np.array([oracle.philox(row[:4], row[4:]) for row in inputs], dtype=np.uint64)
    assert np.array_equal(ours, ref)


def test_output_bits_are_balanced():
    # Each output bit of a good block cipher is 1 half the time.
    blocks = np.array([oracle.philox([i, 7, 0, 0], [1, 0]) for i in range(4096)], dtype=np.uint32)
    bits = np.unpackbits(blocks.view(np.uint8)).reshape(4096, 128)
    frac = bits.mean(axis=0)
    # 4096 samples: sd 0.0078; allow 5 sd
    assert np.all(np.abs(frac - 0.5) < 0.04)
