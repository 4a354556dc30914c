"""Oracle Philox4x32-10 pinned against rocRAND's independent implementation."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND harness")
    exe = str(tmp_path_factory.mktemp("kat") / "rockat")
    subprocess.check_call([hipcc, "-O1", "-o", exe,
                           os.path.join(HERE, "helpers", "rocrand_philox_kat.cpp")],
                          cwd=str(tmp_path_factory.getbasetemp()))

    def run(cases):
        inp = "\n".join(" ".join(str(v) for v in c + k) for c, k in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
        return [[int(t) for t in line.split()] for line in out.stdout.strip().splitlines()]
    return run


def test_philox_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(7)
    cases = [([0, 0, 0, 0], [0, 0]), ([1, 2, 3, 4], [5, 6])]
    for _ in range(200):
        c = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)),  # offset*4 < 2^64
             int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        k = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        cases.append((c, k))
    ref = rocrand_kat(cases)
    for (c, k), r in zip(cases, ref):
        assert O.philox(c, k) == r, (c, k)


def test_philox_words_uniform():
    """Chi-square of the top 8 bits of 2^16 words against uniform."""
    words = []
    for s in range(1 << 14):
        words += O.philox([s, 0, 3, 0], [1, 0])
    top = np.array(words, dtype=np.uint64) >> np.uint64(24)
    counts = np.bincount(top.astype(np.int64), minlength=256)
    exp = len(words) / 256.0
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    # 255 dof: mean 255, sd ~22.6; 5 sigma band
    assert 255 - 5 * 22.6 < chi2 < 255 + 5 * 22.6
