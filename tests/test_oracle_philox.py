"""Pin: the oracle's Philox4x32-10 against rocRAND's open-source engine.

The counter-based stream is the project's reading of the scenario's random
numbers (Sec. III-A, DESPOT: phi = (s0, numbers that determinise the future)).
The block function is checked against an independent implementation, the
host path of rocRAND's header, compiled here from source.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    if shutil.which("hipcc") is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.check_call(["hipcc", "-O2", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe])

    def run(ctr, key):
        ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
        hdr = np.array([key[0], key[1], ctr.shape[0]], dtype=np.uint32)
        p = subprocess.run([exe], input=hdr.tobytes() + ctr.tobytes(), capture_output=True, check=True)
        return np.frombuffer(p.stdout, dtype=np.uint32).reshape(-1, 4)
    return run


def test_philox_matches_rocrand_random_counters(rocrand_ref):
    rng = np.random.default_rng(1234)
    for key in [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (1, 0), (0xA4093822, 0x299F31D0)]:
        ctr = rng.integers(0, 2**32, size=(262144, 4), dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(oracle.philox(ctr, key), rocrand_ref(ctr, key))


def test_philox_matches_rocrand_method_counters(rocrand_ref):
    # counters of the form the method uses: (scenario id, depth, block, tag)
    ids, depth, block, tag = np.meshgrid(np.arange(512), np.arange(96), np.arange(17), np.arange(3),
                                         indexing="ij")
    ctr = np.stack([ids.ravel(), depth.ravel(), block.ravel(), tag.ravel()], 1)
    for key in [(1, 0), (7, 3), (0xDEADBEEF, 41)]:
        assert np.array_equal(oracle.philox(ctr, key), rocrand_ref(ctr, key))


def test_philox_words_look_uniform():
    # a loose sanity check on the output distribution of sequential counters
    ctr = np.zeros((1 << 16, 4), np.uint32)
    ctr[:, 0] = np.arange(1 << 16)
    w = oracle.philox(ctr, (5, 9)).ravel().astype(np.float64) / 2**32
    assert abs(w.mean() - 0.5) < 5 * np.sqrt(1 / 12 / w.size)
    hist = np.bincount((w * 16).astype(int), minlength=16)
    chi2 = ((hist - w.size / 16) ** 2 / (w.size / 16)).sum()
    assert chi2 < 60  # 15 dof; p < 1e-6 beyond this
