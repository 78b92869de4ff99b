"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds input matrices and request traces; it holds none of
the sampler's arithmetic, so both the HIP path's tests/benchmarks and the CPU
oracle's tests draw their inputs from here.

  gaussian_qr    -- U = Q of a QR factorisation of an i.i.d. Gaussian L x N
                    matrix (real, or complex with N(0,1/2) parts): a random
                    delocalised N-fermion Slater determinant (the paper's
                    random wavefunction on a 1D chain, Fig. 3B setting).
  anderson_chain -- lowest-N eigenvectors of a 1D tight-binding chain with
                    hopping -1, open ends and on-site energies uniform in
                    [-W/2, W/2] (the disordered-model setting of the
                    Anderson-Hubbard study, here in 1D); strongly localised.
  dpp_eigvecs    -- eigenvectors of a quality x similarity DPP kernel
                    C_ij = q_i q_j f_i.f_j built from row-normalised Gaussian
                    features (stand-in for the text-summarisation kernel).
"""
import numpy as np


def gaussian_qr(L, N, seed, complex_=False):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((L, N))
    if complex_:
        G = (G + 1j * rng.standard_normal((L, N))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(G)
    return np.ascontiguousarray(Q)


def anderson_chain(L, N, W=2.0, seed=2):
    import scipy.linalg as sl
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-W / 2.0, W / 2.0, L)
    _, V = sl.eigh_tridiagonal(eps, -np.ones(L - 1), select="i",
                               select_range=(0, N - 1))
    # Inverse iteration leaves orthogonality at ~1e-15; a QR keeps the span
    # (the law depends only on the span) and restores it to rounding level.
    Q, R = np.linalg.qr(V)
    Q = Q * np.sign(np.diag(R))[None, :]
    return np.ascontiguousarray(Q)


def dpp_features(L=20000, d=256, seed=4, sigma=0.5):
    """DPP item vectors B = diag(q) F (L x d): F row-normalised Gaussian
    features, quality q ~ LogNormal(0, sigma); the kernel is B B^T."""
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((L, d))
    F /= np.linalg.norm(F, axis=1, keepdims=True)
    q = rng.lognormal(0.0, sigma, L)
    return np.ascontiguousarray(F * q[:, None])


def dpp_eigvecs(L=20000, d=256, seed=4, sigma=0.5):
    """Orthonormal eigenvectors (L x d) and eigenvalues of C = B B^T.

    B from dpp_features; computed on the host through the d x d dual B^T B.
    """
    B = dpp_features(L, d, seed, sigma)
    lam, W = np.linalg.eigh(B.T @ B)
    V = B @ (W / np.sqrt(lam)[None, :])
    Q, R = np.linalg.qr(V)
    Q = Q * np.sign(np.diag(R))[None, :]
    return np.ascontiguousarray(Q), lam


def kdpp_eigen_subset(lam, k, seed):
    """Index set J (|J| = k) of eigenvectors for a k-DPP draw.

    Standard elementary-symmetric-polynomial selection (Kulesza and Taskar's
    DPP review): scan eigenvalues from the last, keep index n with
    probability lam_n e_{l-1}(lam_<n) / e_l(lam_<=n).
    """
    rng = np.random.default_rng(seed)
    lam = np.asarray(lam, dtype=np.float64)
    n = len(lam)
    scale = np.exp(-np.mean(np.log(lam)))   # rescale to avoid overflow
    lam_s = lam * scale
    E = np.zeros((k + 1, n + 1))
    E[0, :] = 1.0
    for l in range(1, k + 1):
        for m in range(1, n + 1):
            E[l, m] = E[l, m - 1] + lam_s[m - 1] * E[l - 1, m - 1]
    J = []
    l = k
    for m in range(n, 0, -1):
        if l == 0:
            break
        if m == l or rng.random() < lam_s[m - 1] * E[l - 1, m - 1] / E[l, m]:
            J.append(m - 1)
            l -= 1
    return sorted(J)


def kdpp_eigen_subsets(lam, k, n, seed):
    """n independent fixed-size eigenvector subsets (int32 [n, k], sorted).

    Same selection as kdpp_eigen_subset -- subset J of size k drawn with
    probability prod_{j in J} lam_j / e_k(lam) -- with the elementary
    symmetric table computed once and all n scans run together.
    """
    rng = np.random.default_rng(seed)
    lam = np.asarray(lam, dtype=np.float64)
    d = len(lam)
    lam_s = lam * np.exp(-np.mean(np.log(lam)))
    E = np.zeros((k + 1, d + 1))
    E[0, :] = 1.0
    for l in range(1, k + 1):
        for m in range(1, d + 1):
            E[l, m] = E[l, m - 1] + lam_s[m - 1] * E[l - 1, m - 1]
    left = np.full(n, k, dtype=np.int64)
    out = np.zeros((n, k), dtype=np.int32)
    for m in range(d, 0, -1):
        act = left > 0
        if not act.any():
            break
        l = np.maximum(left, 1)
        p = lam_s[m - 1] * E[l - 1, m - 1] / E[l, m]
        take = act & ((m == left) | (rng.random(n) < p))
        out[take, left[take] - 1] = m - 1
        left = left - take
    return out


def random_configs(n, k, L, seed, empty_frac=0.0):
    """n rows of k distinct sites in [0, L) (int32); a fraction of the slots
    set to -1 (empty), for estimator tests that need no sampler."""
    rng = np.random.default_rng(seed)
    x = np.stack([rng.choice(L, size=k, replace=False) for _ in range(n)]).astype(np.int32)
    if empty_frac > 0:
        x[rng.random((n, k)) < empty_frac] = -1
    return x


def poisson_trace(rate_hz, duration_s, seed=5,
                  Ls=(1024, 4096, 16384, 65536), Ns=(16, 64, 256, 1024),
                  max_samples=256):
    """Open-loop request trace: arrival time, L, N (N <= L/4), n_samples, seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        L = int(rng.choice(Ls))
        valid = [n for n in Ns if n <= L // 4]
        N = int(rng.choice(valid))
        n = int(rng.integers(1, max_samples + 1))
        out.append({"t": t, "L": L, "N": N, "n": n,
                    "seed": int(rng.integers(0, 2 ** 63))})
    return out
