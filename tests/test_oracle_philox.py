"""Pins the oracle's Philox4x32-10 to rocRAND's philox4x32_10 engine (a library
routine, compiled here for the host) and checks the per-site uniform's bits."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "ref")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(1234)
    cases = []
    for i in range(400):
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] %= 2**30  # the engine maps ctr.xy to a 64-bit offset / 4
        cases.append([int(v) for v in k] + [int(v) for v in c])
    cases += [[0, 0, 0, 0, 0, 0], [2**32 - 1, 2**32 - 1, 2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1],
              [7, 0, 3, 5, 11, 2]]
    inp = "\n".join(" ".join(map(str, c)) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        assert oracle.philox4x32_10(c[2:], c[:2]) == r, c


def test_site_uniform_bits_follow_planes():
    # bit (31 - j) of u is bit (k & 31) of word (k >> 5) & 3 of Philox(k>>7, r, t, 4j + c)
    seed, r, t, c = 0x1234_5678_9ABC, 17, 5, 2
    for k in (0, 31, 32, 77, 127, 128, 300):
        u = oracle.site_uniform(seed, r, k, t, c)
        for j in (0, 1, 13, 31):
            out = oracle.philox4x32_10([k >> 7, r, t, 4 * j + c], [seed & 0xFFFFFFFF, seed >> 32])
            assert (u >> (31 - j)) & 1 == (out[(k >> 5) & 3] >> (k & 31)) & 1


def test_site_uniform_is_uniform():
    # 4096 draws: mean and top-bit balance within loose statistical bounds
    us = np.array([oracle.site_uniform(99, r, k, 3, 1) for r in range(64) for k in range(64)],
                  dtype=np.float64)
    m = us.mean() / 2**32
    assert abs(m - 0.5) < 0.02
    top = (us >= 2**31).mean()
    assert abs(top - 0.5) < 0.04
