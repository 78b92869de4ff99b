"""Pins of the Slater-Jastrow reweighting of the oracle (oracle/jastrow.py):
the reweighted estimate of draws from the exact free law converges to the
brute-force expectation in psi_J; limits and invariances.  CPU only."""
import itertools

import numpy as np

from oracle import jastrow


def _orth(L, N, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((L, N)))
    return q


def _draw_sets(U, n, rng):
    sets = list(itertools.combinations(range(U.shape[0]), U.shape[1]))
    p = np.array([abs(np.linalg.det(U[list(c)])) ** 2 for c in sets])
    idx = rng.choice(len(sets), size=n, p=p / p.sum())
    return np.array([sets[i] for i in idx], dtype=np.int32)


def test_exact_reduces_to_free_marginals():
    # V = 0: <n_i> = diag(U_up U_up^T) + diag(U_dn U_dn^T)
    Uu, Ud = _orth(6, 2, 1), _orth(6, 3, 2)
    dens, D = jastrow.exact(Uu, Ud, 0.0)
    assert np.allclose(dens, (Uu ** 2).sum(1) + (Ud ** 2).sum(1), atol=1e-13)
    # and <D>_0 = sum_i rho_up(i) rho_dn(i) (independent spins)
    assert abs(D - ((Uu ** 2).sum(1) * (Ud ** 2).sum(1)).sum()) < 1e-13


def test_reweighting_converges_to_exact():
    L, V = 6, 1.3
    Uu, Ud = _orth(L, 2, 3), _orth(L, 2, 4)
    ex_dens, ex_D = jastrow.exact(Uu, Ud, V)
    rng = np.random.default_rng(5)
    n = 40000
    xu, xd = _draw_sets(Uu, n, rng), _draw_sets(Ud, n, rng)
    lw, dens, summ = jastrow.estimate(xu, xd, L, V)
    w = np.exp(lw - lw.max())
    _, D = jastrow.log_weights(xu, xd, V)
    # ratio-estimator standard error (delta method)
    for i in range(L):
        o = (xu == i).sum(1) + (xd == i).sum(1)
        r = dens[i]
        se = np.sqrt(((w * (o - r)) ** 2).sum()) / w.sum()
        assert abs(r - ex_dens[i]) < 5 * se + 1e-12, (i, r, ex_dens[i], se)
    se = np.sqrt(((w * (D - summ[0])) ** 2).sum()) / w.sum()
    assert abs(summ[0] - ex_D) < 5 * se
    assert summ[0] < summ[1]          # V > 0 suppresses double occupancy


def test_density_jastrow_matches_gutzwiller_form():
    # v_ij = V/2 delta_ij on total density: sum_i v n_i^2 = V/2 N + V D
    L, V = 5, 0.8
    Uu, Ud = _orth(L, 2, 7), _orth(L, 2, 8)
    d1, D1 = jastrow.exact(Uu, Ud, V)
    d2, D2 = jastrow.exact(Uu, Ud, 0.0, vmat=np.eye(L) * V / 2)
    assert np.allclose(d1, d2, atol=1e-13) and abs(D1 - D2) < 1e-13
    rng = np.random.default_rng(9)
    xu, xd = _draw_sets(Uu, 50, rng), _draw_sets(Ud, 50, rng)
    l1, e1, s1 = jastrow.estimate(xu, xd, L, V)
    l2, e2, s2 = jastrow.estimate(xu, xd, L, 0.0, vmat=np.eye(L) * V / 2)
    assert np.allclose(l1 - l2, V / 2 * 4)       # constant N = 4 offset
    assert np.allclose(e1, e2, atol=1e-13)


def test_shift_invariance_and_empty_slots():
    rng = np.random.default_rng(11)
    xu = np.array([[0, 2, -1], [1, 3, 4], [2, -1, -1]], dtype=np.int32)
    xd = np.array([[2, 4], [1, 0], [3, 2]], dtype=np.int32)
    a = jastrow.estimate(xu, xd, 5, 0.7)
    b = jastrow.estimate(xu, xd, 5, 0.7, extra=np.full(3, 123.0))
    assert np.allclose(a[1], b[1]) and np.allclose(a[2][:2], b[2][:2])
    lw, D = jastrow.log_weights(xu, xd, 0.7)
    assert list(D) == [1, 1, 1]
    # density sums to the mean reweighted particle number
    w = np.exp(a[0] - a[0].max())
    nparts = (xu >= 0).sum(1) + (xd >= 0).sum(1)
    assert abs(a[1].sum() - (w * nparts).sum() / w.sum()) < 1e-13
