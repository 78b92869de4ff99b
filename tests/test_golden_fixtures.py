"""The stored oracle results under tests/golden/ are the oracle's: a few rows
recomputed here with oracle/ must reproduce them, their log-determinants
must equal log|det U[x, :]|^2 (Eq. (1)), every row is a valid configuration,
and the input probe matches the seeded generator.  CPU only."""
import os

import numpy as np
import pytest

from oracle import sampler
from paper_2109_07358_amd import workloads

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    z = np.load(os.path.join(HERE, name + ".npz"))
    return {k: z[k] for k in z.files}


@pytest.fixture(scope="module")
def c2():
    return load("c2_chain_L4096_N256"), workloads.anderson_chain(4096, 256, 2.0, 2)


@pytest.fixture(scope="module")
def c3():
    return load("c3_complex_L16384_N512"), workloads.gaussian_qr(16384, 512, 3, complex_=True)


def _common(g, U):
    L, N = U.shape
    assert int(g["L"]) == L and int(g["N"]) == N
    assert np.max(np.abs(U[g["probe_rows"]] - g["probe"])) < 1e-10
    X = g["sites"].astype(np.int64)
    assert X.shape == (len(g["samples"]), N)
    assert X.min() >= 0 and X.max() < L
    assert all(len(np.unique(r)) == N for r in X[:: max(1, len(X) // 64)])
    m = g["near_margin"]
    assert np.all((m >= 0) & (m < 1e-6))
    assert np.all(g["min_margin"] > 0)
    for i in (0, len(X) // 2, len(X) - 1):
        _, l = np.linalg.slogdet(U[X[i]])
        assert abs(g["logdet"][i] - 2 * l) < 1e-9 * max(1.0, abs(l))
    return X


def test_chain_fixture_is_the_oracles(c2):
    g, U = c2
    X = _common(g, U)
    assert len(X) == 3 * 4096 and np.array_equal(g["samples"], np.arange(3 * 4096))
    for i in (0, 4096, 12287):
        r = sampler.sample_one(U, int(g["seed"]), int(g["samples"][i]))
        assert np.array_equal(r["x"], X[i])
        assert r["logdet"] == g["logdet"][i]
        listed = {int(k): m for (j, k), m in zip(g["near_idx"], g["near_margin"]) if j == i}
        for k, m in enumerate(r["margin"]):
            if m < 1e-6:
                assert listed[k] == m


def test_complex_fixture_is_the_oracles(c3):
    g, U = c3
    X = _common(g, U)
    assert len(X) == 32
    r = sampler.sample_one(U, int(g["seed"]), int(g["samples"][5]), 24)
    assert np.array_equal(r["x"], X[5][:24])
