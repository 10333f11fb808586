"""Pins of the oracle's Philox4x32-10 (Salmon et al., SC'11).

The witness is rocRAND's open-source philox4x32_10 engine, compiled here as
host code from its header; it shares nothing with the oracle.  Statistical
checks guard against a mistake that would keep both in agreement only by
accident (they cannot: the witness is an independent implementation)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
WITNESS_SRC = os.path.join(HERE, "witness", "philox_witness.cpp")


@pytest.fixture(scope="module")
def witness(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND witness")
    exe = str(tmp_path_factory.mktemp("w") / "philox_witness")
    subprocess.run([hipcc, "-O1", "-o", exe, WITNESS_SRC], check=True,
                   cwd=str(tmp_path_factory.getbasetemp()))

    def run(rows):
        txt = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=txt, capture_output=True, text=True,
                             check=True).stdout
        return np.array([[int(t) for t in ln.split()] for ln in
                         out.strip().splitlines()], dtype=np.uint64)

    return run


def test_philox_matches_rocrand_witness(witness):
    rng = np.random.default_rng(12345)
    rows = []
    # key and counter words over their full ranges; counter word 1 is kept
    # below 2^30 so the witness can reach it through its offset argument
    for _ in range(300):
        k0, k1 = rng.integers(0, 2**32, 2)
        c0, c2, c3 = rng.integers(0, 2**32, 3)
        c1 = rng.integers(0, 2**30)
        rows.append((k0, k1, c0, c1, c2, c3))
    rows += [(0, 0, 0, 0, 0, 0), (1, 0, 0, 0, 0, 0),
             (2**32 - 1, 2**32 - 1, 2**32 - 1, 2**30 - 1, 2**32 - 1,
              2**32 - 1)]
    want = witness(rows)
    for r, w in zip(rows, want):
        got = oracle.philox4x32_10([r[2], r[3], r[4], r[5]], [r[0], r[1]])
        assert got.astype(np.uint64).tolist() == w.tolist(), r


def _block(c0, c1, c2, c3, k0=7, k1=9):
    return oracle.philox4x32_10([c0, c1, c2, c3], [k0, k1])


def test_every_input_word_matters():
    base = _block(1, 2, 3, 4)
    for i in range(6):
        args = [1, 2, 3, 4, 7, 9]
        args[i] ^= 1
        assert not np.array_equal(_block(*args), base), i


def test_output_bits_balanced_and_uniform():
    words = np.concatenate([_block(c, 5, 11, 0) for c in range(20000)])
    bits = (words[:, None] >> np.arange(32, dtype=np.uint32)) & 1
    frac = bits.mean(axis=0)
    sigma = np.sqrt(0.25 / len(words))
    assert np.all(np.abs(frac - 0.5) < 5 * sigma)
    # chi^2 of the top byte over 256 cells: mean 255, sd ~22.6
    cnt = np.bincount((words >> 24).astype(np.int64), minlength=256)
    expect = len(words) / 256
    chi2 = ((cnt - expect) ** 2 / expect).sum()
    assert 255 - 5 * 22.6 < chi2 < 255 + 5 * 22.6
