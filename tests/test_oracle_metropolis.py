"""Pins of the Metropolis conditional update of the oracle
(oracle/metropolis.py): with enough iterations its law is the determinant
law (brute force, chi-square), its one-step chains target the conditional
weights, and its configurations are always valid.  CPU only."""
import itertools
import math

import numpy as np
import pytest

from oracle import brute, metropolis, sampler


def _orth(L, N, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((L, N)))
    return q


def _chi2_sets(U, draws):
    law = brute.set_law(brute.det_law(U))
    keys = sorted(law)
    n = len(draws)
    counts = {k: 0 for k in keys}
    for x in draws:
        counts[tuple(sorted(x))] += 1
    exp = np.array([law[k] * n for k in keys])
    obs = np.array([counts[k] for k in keys])
    keep = exp > 5
    chi2 = float((((obs - exp) ** 2) / exp)[keep].sum())
    return chi2, int(keep.sum()) - 1


@pytest.mark.parametrize("radius,m_cond", [(0, 60), (2, 200)])
def test_long_chains_reach_the_determinant_law(radius, m_cond):
    # local moves mix more slowly (low-weight sites sit between the modes)
    U = _orth(7, 2, 3)
    draws = [metropolis.sample_one_mh(U, 17, s, m_cond, radius)["x"] for s in range(3000)]
    chi2, dof = _chi2_sets(U, draws)
    # P(chi2 > dof + 6 sqrt(2 dof)) is far below 1e-3 for these dof
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


def test_first_step_targets_the_conditional():
    # N = 1: the conditional of the only step is |U[y, 0]|^2
    U = _orth(9, 1, 5)
    p = U[:, 0] ** 2
    n = 4000
    counts = np.zeros(9)
    for s in range(n):
        counts[metropolis.sample_one_mh(U, 23, s, 40, 0)["x"][0]] += 1
    chi2 = float(((counts - n * p) ** 2 / (n * p)).sum())
    assert chi2 < 8 + 6 * 4, chi2


def test_configurations_are_valid_and_column_order_shared():
    U = _orth(12, 5, 7)
    for s in range(30):
        r = metropolis.sample_one_mh(U, 5, s, 3, 1)
        assert len(set(r["x"])) == 5 and all(0 <= y < 12 for y in r["x"])
        assert r["m"] == sampler.column_order(5, s, 5)
        # logdet = log |det U[x, m]|^2 of the drawn configuration
        _, l = np.linalg.slogdet(U[np.array(r["x"])][:, r["m"]])
        assert abs(r["logdet"] - 2 * l) < 1e-9


def test_zero_iterations_stay_at_the_anchor_or_nearest_site():
    U = _orth(10, 3, 9)
    anchor = [int(np.argmax(U[:, c] ** 2)) for c in range(3)]
    r = metropolis.sample_one_mh(U, 1, 0, 0, 0)
    xs = []
    for t, y in enumerate(r["x"]):
        w = sampler.conditional_weights(U, xs, r["m"][: t + 1])
        a = anchor[r["m"][t]]
        if w[a] > 0:
            assert y == a
        else:
            d = abs(y - a)
            assert w[y] > 0 and all(w[z] == 0 for z in range(10) if abs(z - a) < d)
        xs.append(y)
