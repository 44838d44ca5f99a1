"""Pin of the oracle's Philox4x32-10 against an independent implementation:
rocRAND's header engine, compiled for the host and run (not copied) here.
Skipped when hipcc or the rocRAND headers are missing."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

PROBE = os.path.join(os.path.dirname(__file__), "golden", "philox_rocrand_probe.cpp")


@pytest.fixture(scope="module")
def probe_exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "probe")
    subprocess.check_call([hipcc, "-O1", "-o", exe, PROBE], cwd=d)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_bit_exact_vs_rocrand(probe_exe):
    rng = np.random.default_rng(2024)
    cases = rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64)
    cases[:4] = 0
    cases[1, :4] = [0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]
    cases[2, 4:] = [0xFFFFFFFF, 0xFFFFFFFF]
    cases[3, :] = [7, 0, 1002, 0, 1002, 0]
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    out = subprocess.run([probe_exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()], np.uint64)
    for row, r in zip(cases, ref):
        got = oracle.philox(row[:4].astype(np.uint32), row[4:].astype(np.uint32))
        assert np.array_equal(got.astype(np.uint64), r), (row, got, r)
