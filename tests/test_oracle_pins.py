"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: every check is against an
independent quantity -- the Eq. (1) law by enumeration, literal determinants,
closed forms that orthonormality implies, slogdet, an independent Philox
implementation (rocRAND, compiled on the host), brute-force loops and
chi-square statistics.  The planted-mistake tests show that plausible
mistakes in the oracle's arithmetic fail these pins.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import brute, philox, sampler
from paper_2109_07358_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------- Philox --
@pytest.fixture(scope="module")
def rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "probe")
    r = subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                        os.path.join(HERE, "rocrand_philox_probe.cpp"),
                        "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("rocRAND probe did not build: " + r.stderr[-400:])
    return exe


def test_philox_matches_rocrand(rocrand_probe):
    # rocRAND keys Philox with (seed lo, seed hi), puts the subsequence in
    # counter words 2,3 and offset/4 in words 0,1: our counter
    # (sample lo, sample hi, step, 0) is subsequence=step, offset=4*sample.
    cases = [(0, 0, 0), (0x5EED, 3, 17), (2 ** 63 + 12345, 2 ** 40 + 7, 255),
             (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFF, 511), (42, 123456789, 1023)]
    args = []
    for seed, s, t in cases:
        args += [str(seed), str(t), str(4 * s)]
    out = subprocess.run([rocrand_probe] + args, capture_output=True,
                         text=True, check=True).stdout.split("\n")
    for (seed, s, t), line in zip(cases, out):
        want = tuple(int(v) for v in line.split())
        assert philox.step_words(seed, s, t) == want


def test_fisher_yates_index_exact():
    rng = np.random.default_rng(0)
    for _ in range(200):
        w = tuple(int(v) for v in rng.integers(0, 2 ** 32, 4))
        n = int(rng.integers(1, 5000))
        t = int(rng.integers(0, n))
        j = philox.fisher_yates_index(w, t, n)
        v = (w[1] << 32) | w[0]
        assert t <= j < n
        # floor(v * R / 2^64) by exact rational arithmetic
        assert j - t == (v * (n - t)) // (1 << 64)


def test_fisher_yates_gives_uniform_permutations():
    N, n = 4, 24000
    counts = {}
    for s in range(n):
        p = tuple(sampler.column_order(7, s, N))
        counts[p] = counts.get(p, 0) + 1
    assert len(counts) == math.factorial(N)
    obs = np.array(list(counts.values()))
    assert stats.chisquare(obs).pvalue > 1e-4


def test_uniform53_is_53_bit_dyadic():
    for s in range(50):
        u = philox.uniform53(philox.step_words(1, s, 3))
        assert 0.0 <= u < 1.0
        assert float(u * 2 ** 53).is_integer()
    assert philox.uniform53((0, 0, 0xFFFFFFFF, 0xFFFFFFFF)) == 1.0 - 2.0 ** -53
    assert philox.uniform53((0, 0, 0, 0)) == 0.0


# ------------------------------------------------------------ Eq. (1)/(2) --
def _cases():
    return [("real_8x3", workloads.gaussian_qr(8, 3, 1)),
            ("cplx_7x3", workloads.gaussian_qr(7, 3, 11, complex_=True)),
            ("real_6x4", workloads.gaussian_qr(6, 4, 12))]


@pytest.mark.parametrize("name,U", _cases())
def test_cauchy_binet(name, U):
    assert abs(brute.cauchy_binet_total(U) - 1.0) < 1e-12


@pytest.mark.parametrize("name,U", _cases())
def test_sampler_law_is_det_law(name, U):
    """Eq. (2): averaging the chain of conditionals over m gives Eq. (1)."""
    want = brute.det_law(U)
    got = brute.sampler_law(U)
    assert abs(sum(got.values()) - 1.0) < 1e-12
    err = max(abs(got.get(x, 0.0) - p) for x, p in want.items())
    assert err < 1e-12
    assert set(got) <= set(want)


# -------------------------------------------------- Eq. (3) weights, SI S-1 --
@pytest.mark.parametrize("cplx", [False, True])
def test_schur_weights_match_determinants(cplx):
    U = workloads.gaussian_qr(10, 4, 21, complex_=cplx)
    rng = np.random.default_rng(3)
    for _ in range(20):
        k = int(rng.integers(1, 5))
        cols = list(rng.permutation(4)[:k])
        xs = list(rng.choice(10, k - 1, replace=False))
        a = sampler.conditional_weights(U, xs, cols)
        b = sampler.conditional_weights_det(U, xs, cols)
        assert np.allclose(a, b, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("cplx", [False, True])
def test_weight_total_closed_form(cplx):
    # sum_y |v(y)|^2 = |Gamma|^2 = 1 + |beta|^2 for orthonormal columns, and
    # v vanishes on the conditioning rows (h is normal to them).
    U = workloads.gaussian_qr(64, 16, 5, complex_=cplx)
    rng = np.random.default_rng(4)
    for k in (1, 2, 8, 16):
        cols = list(rng.permutation(16)[:k])
        xs = list(rng.choice(64, k - 1, replace=False))
        v, beta = sampler.conditional_amplitudes(U, xs, cols)
        tot = float(np.sum(np.abs(v) ** 2))
        assert abs(tot - (1.0 + float(np.sum(np.abs(beta) ** 2)))) < 1e-10 * tot
        if xs:
            assert np.max(np.abs(v[xs])) < 1e-10 * math.sqrt(tot)
        w = sampler.conditional_weights(U, xs, cols)
        assert np.all(w[xs] == 0.0)


def test_first_step_closed_form():
    U = workloads.gaussian_qr(32, 5, 6)
    for m1 in range(5):
        w = sampler.conditional_weights(U, [], [m1])
        assert np.array_equal(w, U[:, m1] ** 2)


@pytest.mark.parametrize("cplx", [False, True])
def test_logdet_identity(cplx):
    # prod_k |s_k|^2 = |det U[x, m]|^2 = |det U[x, :]|^2 (Schur complements)
    U = workloads.gaussian_qr(64, 16, 8, complex_=cplx)
    for s in range(5):
        r = sampler.sample_one(U, 99, s)
        _, ld = np.linalg.slogdet(U[r["x"], :])
        assert abs(r["logdet"] - 2.0 * ld) < 1e-9 * max(1.0, abs(ld))
        assert len(set(r["x"])) == 16


def test_marginal_is_prefix():
    U = workloads.gaussian_qr(64, 16, 9)
    full, _, _ = sampler.sample(U, 5, 10, 20)
    part, _, _ = sampler.sample(U, 5, 10, 20, n_keep=6)
    assert np.array_equal(full[:, :6], part)


# ------------------------------------------------------------- the draw --
def _first_exceeding(w, u):
    T = 0.0
    for v in w:
        T += v
    target = u * T
    run = 0.0
    for i, v in enumerate(w):
        run += v
        if run > target:
            return i
    raise AssertionError


def test_inverse_cdf_bruteforce():
    rng = np.random.default_rng(10)
    for _ in range(300):
        L = int(rng.integers(1, 40))
        w = rng.random(L) * (rng.random(L) < 0.7)
        if w.sum() == 0:
            w[int(rng.integers(0, L))] = 1.0
        u = float(rng.random())
        x, T, margin = sampler.inverse_cdf(w, u)
        assert x == _first_exceeding(w, u)
        assert w[x] > 0 and margin >= 0.0
    # edge cases: u = 0 skips leading zero-weight sites; u -> 1 picks the last
    # non-zero site even when trailing sites are zero.
    assert sampler.inverse_cdf(np.array([0.0, 0.0, 1.0, 1.0]), 0.0)[0] == 2
    assert sampler.inverse_cdf(np.array([1.0, 1.0, 0.0]), 1 - 2 ** -53)[0] == 1
    with pytest.raises(FloatingPointError):
        sampler.inverse_cdf(np.zeros(4), 0.5)


# ------------------------------------------------------------- statistics --
def test_chisquare_subset_histogram():
    """The oracle's samples follow the Eq. (1) set law (L=8, N=3)."""
    U = workloads.gaussian_qr(8, 3, 1)
    law = brute.set_law(brute.det_law(U))
    keys = sorted(law)
    X, _, _ = sampler.sample(U, 0x5EED, 0, 40000)
    idx = {k: i for i, k in enumerate(keys)}
    obs = np.zeros(len(keys))
    for row in X:
        obs[idx[tuple(sorted(row))]] += 1
    exp = np.array([law[k] for k in keys]) * len(X)
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def test_site_marginals_match_density():
    """Site occupation frequency -> diag(U U^T); sum of marginals = N."""
    U = workloads.gaussian_qr(64, 16, 0)
    rho = sampler.density(U)
    assert abs(rho.sum() - 16) < 1e-12
    n = 2000
    X, _, _ = sampler.sample(U, 3, 0, n)
    freq = np.bincount(X.ravel(), minlength=64) / n
    z = (freq - rho) / np.sqrt(rho * (1 - rho) / n)
    assert np.max(np.abs(z)) < 5.0


# ------------------------------------------------------- planted mistakes --
def _mutant(kind):
    def fn(U, xs, cols):
        cols = [int(c) for c in cols]
        xs = [int(x) for x in xs]
        if len(cols) == 1:
            v = U[:, cols[0]].copy()
        else:
            A = U[np.ix_(xs, cols[:-1])]
            c = U[xs, cols[-1]]
            if kind == "transposed":
                beta = np.linalg.solve(A.T, c)
            elif kind == "conjugated":
                beta = np.linalg.solve(A.conj(), c)
            else:
                beta = np.linalg.solve(A, c)
            if kind == "dropped_term":
                v = U[:, cols[-1]].copy()
            elif kind == "wrong_sign":
                v = U[:, cols[-1]] + U[:, cols[:-1]] @ beta
            elif kind == "wrong_index":
                v = U[:, cols[-1]] - U[:, cols[:-1][::-1]] @ beta
            else:
                v = U[:, cols[-1]] - U[:, cols[:-1]] @ beta
        w = np.abs(v) ** 2
        if kind != "unmasked":
            w[xs] = 0.0
        return w
    return fn


@pytest.mark.parametrize("kind", ["dropped_term", "wrong_sign", "wrong_index",
                                  "transposed", "conjugated"])
def test_planted_mistakes_fail_the_law_pin(kind):
    U = (workloads.gaussian_qr(7, 3, 11, complex_=True) if kind == "conjugated"
         else workloads.gaussian_qr(8, 3, 1))
    want = brute.det_law(U)
    got = brute.sampler_law(U, weight_fn=_mutant(kind))
    err = max(abs(got.get(x, 0.0) - p) for x, p in want.items())
    assert err > 1e-6, kind


def test_planted_shared_column_order_fails_the_law_pin():
    # A single fixed order m (no per-sample permutation) gives the wrong law.
    U = workloads.gaussian_qr(8, 3, 1)
    L, N = U.shape
    law = {}

    def rec(xs, p):
        if len(xs) == N:
            law[tuple(xs)] = p
            return
        w = sampler.conditional_weights(U, xs, list(range(len(xs) + 1)))
        w = w / w.sum()
        for y in range(L):
            if w[y] > 0:
                rec(xs + [y], p * w[y])
    rec([], 1.0)
    want = brute.set_law(brute.det_law(U))
    got = brute.set_law(law)
    assert max(abs(got.get(k, 0) - v) for k, v in want.items()) > 1e-3
