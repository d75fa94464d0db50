"""Pin of the oracle's Philox4x32-10 against an independent implementation.

The oracle's generator (Salmon et al., SC'11) is compared word for word with
rocRAND's Philox4x32-10 engine, compiled from ROCm's headers and run on the
host CPU, on random counters and keys plus the edge cases of 32-bit carries.
rocRAND is a separate code base, so a wrong constant, a swapped word or a
missing key bump in the oracle fails here.  Parity: pinned.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_dump(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_dump")
    subprocess.run([hipcc, "-O2", os.path.join(HERE, "helpers", "rocrand_philox_dump.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


def _cases(n, seed):
    rng = np.random.default_rng(seed)
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    edge = np.array([[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 0, 0, 1 << 24],
                     [0xFFFFFFFF, 0, 0, 0], [5, 7, 3, (6 << 24) | 2]], dtype=np.uint32)
    ekey = np.array([[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [1, 0], [0, 1], [63, 0], [7, 0]],
                    dtype=np.uint32)
    return np.vstack([edge, ctr]), np.vstack([ekey, key])


def test_philox_matches_rocrand(rocrand_dump):
    ctr, key = _cases(200_000, 1234)
    lines = "\n".join(f"{c[0]:x} {c[1]:x} {c[2]:x} {c[3]:x} {k[0]:x} {k[1]:x}"
                      for c, k in zip(ctr, key))
    res = subprocess.run([rocrand_dump], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(t, 16) for t in ln.split()] for ln in res.stdout.splitlines()],
                   dtype=np.uint64).astype(np.uint32)
    got = oracle.philox(ctr, key)
    assert ref.shape == got.shape
    bad = np.nonzero(np.any(ref != got, axis=1))[0]
    assert bad.size == 0, f"first mismatch at case {bad[:5]}"


def test_philox_is_a_bijection_on_a_sample():
    # distinct counters under one key give distinct outputs (a permutation)
    ctr = np.zeros((100_000, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(100_000)
    out = oracle.philox(ctr, np.zeros((100_000, 2), dtype=np.uint32))
    v = out.view(np.dtype((np.void, 16))).ravel()
    assert np.unique(v).size == 100_000
    # words are uniform: mean of the top bit of every word ~ 1/2
    bits = (out >> 31).astype(np.float64)
    assert abs(bits.mean() - 0.5) < 5 * 0.5 / np.sqrt(bits.size)
