"""Pins of the oracle's noise realisation: Philox4x32-10 words against rocRAND's
engine (a library routine, compiled here for the host), the Box-Muller pairing
identities and the normal law (Kolmogorov-Smirnov against scipy)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_ref.cpp")


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("ph") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, HELPER])

    def run(ctr, key):
        out = subprocess.check_output([exe, *[str(int(c)) for c in ctr], *[str(int(k)) for k in key]])
        return np.array([int(t) for t in out.split()], np.uint32)
    return run


def test_philox_words_match_rocrand(oracle, rocrand_ref):
    rng = np.random.default_rng(0)
    cases = [([0, 0, 0, 0], [0, 0]), ([1, 0, 0, 0], [0, 0]), ([0, 5, 0, 0], [7, 0])]
    for _ in range(12):
        ctr = [rng.integers(0, 2**32), rng.integers(0, 2**29), rng.integers(0, 2**32),
               rng.integers(0, 2**32)]
        cases.append((ctr, [rng.integers(0, 2**32), rng.integers(0, 2**32)]))
    for ctr, key in cases:
        assert np.array_equal(oracle.philox(ctr, key), rocrand_ref(ctr, key)), (ctr, key)


def test_box_muller_pairing(oracle):
    """Normals 0,1 (2,3) of a counter are the cos/sin pair of words 0,1 (2,3):
    z0^2 + z1^2 = -2 ln u0 and atan2(z1, z0) = 2 pi u1 (mod 2 pi)."""
    for seed, inst, blk, k in [(0, 0, 0, 0), (3, 17, 1234, 5), (9, 4095, 25000, 67)]:
        w = oracle.philox([blk, k, 0, 0], [seed, inst]).astype(np.float64)
        u = (w + 0.5) / 2.0**32
        z = [oracle.normal(seed, inst, 4 * blk + q, k) for q in range(4)]
        for p in range(2):
            np.testing.assert_allclose(z[2 * p] ** 2 + z[2 * p + 1] ** 2, -2 * np.log(u[2 * p]),
                                       rtol=1e-12)
            ang = np.mod(np.arctan2(z[2 * p + 1], z[2 * p]), 2 * np.pi)
            np.testing.assert_allclose(ang, 2 * np.pi * u[2 * p + 1], rtol=0, atol=1e-9)


def test_normals_are_standard_normal(oracle):
    z = np.array([oracle.normal(0, i % 97, n, i // 97) for i in range(200) for n in range(400)])
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # consecutive steps of one region are uncorrelated
    s = np.array([oracle.normal(1, 2, n, 3) for n in range(20000)])
    assert abs(np.corrcoef(s[1:], s[:-1])[0, 1]) < 0.03
