"""CPU checks of the seeded input generators (shared by the oracle tests and
the GPU tests, holding none of the sampler's arithmetic)."""
import itertools
from collections import Counter

import numpy as np
from scipy import stats

from paper_2109_07358_amd import workloads


def test_gaussian_qr_orthonormal():
    for c in (False, True):
        U = workloads.gaussian_qr(200, 30, 1, complex_=c)
        assert np.allclose(U.conj().T @ U, np.eye(30), atol=1e-12)


def test_anderson_chain_is_lowest_eigenvectors():
    L, N, W = 300, 20, 2.0
    U = workloads.anderson_chain(L, N, W, 2)
    assert np.allclose(U.T @ U, np.eye(N), atol=1e-12)
    rng = np.random.default_rng(2)
    eps = rng.uniform(-W / 2, W / 2, L)
    H = np.diag(eps) - np.eye(L, k=1) - np.eye(L, k=-1)
    w = np.linalg.eigvalsh(H)
    # U spans the lowest-N eigenspace: U^T H U has the N lowest eigenvalues
    assert np.allclose(np.sort(np.linalg.eigvalsh(U.T @ H @ U)), w[:N], atol=1e-9)


def test_kdpp_subsets_follow_the_product_law():
    lam = np.array([0.5, 1.0, 2.0, 3.0, 0.7, 1.5])
    k, n = 3, 200000
    J = workloads.kdpp_eigen_subsets(lam, k, n, 1)
    assert J.shape == (n, k) and (np.diff(J, axis=1) > 0).all()
    subs = list(itertools.combinations(range(len(lam)), k))
    p = np.array([np.prod(lam[list(s)]) for s in subs])
    p /= p.sum()
    c = Counter(map(tuple, J))
    obs = np.array([c[s] for s in subs])
    chi2 = ((obs - n * p) ** 2 / (n * p)).sum()
    assert stats.chi2.sf(chi2, len(subs) - 1) > 1e-3


def test_dpp_eigvecs_orthonormal_with_positive_spectrum():
    V, lam = workloads.dpp_eigvecs(2000, 32, 4)
    assert np.allclose(V.T @ V, np.eye(32), atol=1e-12)
    assert (lam > 0).all()


def test_poisson_trace_shapes():
    tr = workloads.poisson_trace(2000.0, 0.5, 5)
    assert 800 < len(tr) < 1200
    for r in tr:
        assert r["N"] <= r["L"] // 4 and 1 <= r["n"] <= 256
