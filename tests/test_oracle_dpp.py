"""Pins of the DPP front end of the oracle (oracle/dpp.py) to closed forms,
brute force and the exact selection laws.  CPU only."""
import itertools
import math

import numpy as np
import pytest

from oracle import dpp, philox


def _orth(L, d, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((L, d)))
    return q


def test_dual_eig_closed_form():
    # B = Q diag(s) R^T with Q (L x d), R (d x d) orthogonal: B B^T has
    # eigenvalues s^2 with eigenvectors the columns of Q.
    L, d = 40, 6
    Q = _orth(L, d, 1)
    R = _orth(d, d, 2)
    s = np.array([0.5, 1.0, 1.5, 2.0, 3.0, 4.5])
    B = Q @ np.diag(s) @ R.T
    lam, U, W = dpp.dual_eig(B)
    assert np.allclose(lam, s ** 2, rtol=1e-13)
    # columns of U equal the columns of Q up to sign, in ascending s
    for j in range(d):
        assert abs(abs(U[:, j] @ Q[:, j]) - 1.0) < 1e-12


def test_dual_eig_invariants():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((30, 5)) * rng.lognormal(0, 0.5, 30)[:, None]
    lam, U, W = dpp.dual_eig(B)
    C = B @ B.T
    assert np.abs(C @ U - U * lam[None, :]).max() < 1e-11 * lam.max()
    assert np.abs(U.T @ U - np.eye(5)).max() < 1e-13
    assert abs(lam.sum() - (B ** 2).sum()) < 1e-12 * lam.sum()   # trace
    assert np.all(np.diff(lam) > 0)
    for j in range(5):
        r = int(np.argmax(np.abs(W[:, j])))
        assert W[r, j] > 0


def test_esp_table_brute_force():
    lam = np.array([0.3, 1.7, 0.9, 2.5, 1.1, 0.05])
    k = 4
    E = dpp.esp_table(lam, k)
    mu = lam / lam.max()
    for j in range(len(lam) + 1):
        for m in range(k + 1):
            want = sum(math.prod(mu[list(c)]) for c in itertools.combinations(range(j), m))
            assert abs(E[m][j] - want) <= 1e-14 * max(1.0, want)


def test_kdpp_law():
    # subset J of size k with probability prod lam_J / e_k(lam)
    lam = np.array([0.4, 1.3, 2.0, 0.7, 1.0])
    k = 2
    E = dpp.esp_table(lam, k)
    subsets = list(itertools.combinations(range(5), k))
    p = np.array([math.prod(lam[list(J)]) for J in subsets])
    p /= p.sum()
    n = 20000
    counts = {J: 0 for J in subsets}
    for s in range(n):
        J = tuple(dpp.kdpp_select(lam, k, 11, s, E=E))
        assert len(J) == k
        counts[J] += 1
    obs = np.array([counts[J] for J in subsets])
    chi2 = float(((obs - n * p) ** 2 / (n * p)).sum())
    # 9 degrees of freedom: P(chi2 > 33.7) < 1e-4
    assert chi2 < 33.7, chi2


def test_kdpp_forced_and_full():
    lam = np.array([0.2, 0.9, 3.0])
    assert dpp.kdpp_select(lam, 3, 5, 0) == [0, 1, 2]
    # a zero eigenvalue is never kept when k <= number of nonzero ones
    lam0 = np.array([0.0, 1.0, 2.0, 0.5])
    for s in range(200):
        assert 0 not in dpp.kdpp_select(lam0, 3, 9, s)


def test_dpp_law():
    lam = np.array([0.1, 1.0, 4.0, 9.0])
    n = 20000
    hits = np.zeros(4)
    sizes = []
    for s in range(n):
        J = dpp.dpp_select(lam, 13, s)
        assert J == sorted(J)
        for j in J:
            hits[j] += 1
        sizes.append(len(J))
    p = lam / (lam + 1.0)
    sd = np.sqrt(n * p * (1 - p))
    assert np.all(np.abs(hits - n * p) < 5 * sd + 1)
    assert abs(np.mean(sizes) - p.sum()) < 5 * np.sqrt((p * (1 - p)).sum() / n)


def test_selection_stream_is_not_the_sampler_stream():
    assert philox.stream_words(7, 3, 2, 1) != philox.step_words(7, 3, 2)
    assert philox.stream_words(7, 3, 2, 0) == philox.step_words(7, 3, 2)
