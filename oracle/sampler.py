"""The FFS sampler, written plainly from the paper (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Problem (Eq. (1)): U is L x N with orthonormal columns; an ordered
configuration x = (x_1..x_N) of distinct sites has probability
|det U[x, :]|^2 / N!.

Method (Eq. (2) and the conditional defined right after it): draw a uniformly
random column order m, then for k = 1..N draw x_k from the conditional whose
weight over candidate sites y is |det U[(x_<k, y), m_<=k]|^2, normalised over
y.  Eq. (3) / SI S-1 (geometrical approach): that determinant equals the
fixed base volume |det U[x_<k, m_<k]|^2 times |u_y^T h|^2, where u_y is the
row U[y, m_<=k] and h is a normal vector to the k-1 rows u_{x_1..x_{k-1}}.
With h = (-beta, 1), beta solving U[x_<k, m_<k] beta = U[x_<k, m_k], the
unnormalised weight is |v(y)|^2 with v = U[:, m_k] - U[:, m_<k] beta.  For
complex U, "perpendicular" is read bilinearly (u^T h, no conjugate, as the
paper writes the transpose), which keeps |u^T h|^2 proportional to |det|^2.

Readings of points the paper leaves open (same on the GPU side):
  * weights are normalised over the L-k+1 free sites; occupied sites get
    weight exactly 0 and can never be drawn (SI S-1 counts L-k+1 candidates);
  * m is drawn independently per sample (lazy Fisher-Yates, see philox.py);
  * the draw is the inverse CDF over ascending site index: x_k is the first
    site whose running sum F exceeds u*T, T being the computed total;
  * beta is solved afresh at every step with LAPACK (partial pivoting); the
    paper's iterative elimination (SI S-1) is an optimisation of the same
    quantity and is not reproduced here;
  * positions are 0-based and returned in draw order.
"""
import numpy as np

from . import philox


def _abs2(v):
    if np.iscomplexobj(v):
        return v.real * v.real + v.imag * v.imag
    return v * v


def conditional_amplitudes(U, xs, cols):
    """v(y) = u_y^T h for all sites y (Eq. (3)), with h = (-beta, 1).

    xs: the k-1 sites already drawn; cols: m_1..m_k (k column indices).
    Returns (v, beta); beta has length k-1.
    """
    cols = [int(c) for c in cols]
    xs = [int(x) for x in xs]
    k = len(cols)
    if k == 1:
        return U[:, cols[0]].copy(), np.zeros(0, dtype=U.dtype)
    A = U[np.ix_(xs, cols[:-1])]
    c = U[xs, cols[-1]]
    beta = np.linalg.solve(A, c)
    v = U[:, cols[-1]] - U[:, cols[:-1]] @ beta
    return v, beta


def conditional_weights(U, xs, cols):
    """Unnormalised conditional weights |u_y^T h|^2, occupied sites zeroed."""
    v, _ = conditional_amplitudes(U, xs, cols)
    w = _abs2(v)
    w[[int(x) for x in xs]] = 0.0
    return w


def conditional_weights_det(U, xs, cols):
    """Same weights from literal determinants (Eq. (2)'s conditional).

    |det U[(x_<k, y), m_<=k]|^2 / |det U[x_<k, m_<k]|^2 for every y.  O(L k^3);
    for tiny cases only.
    """
    cols = [int(c) for c in cols]
    xs = [int(x) for x in xs]
    L = U.shape[0]
    base = abs(np.linalg.det(U[np.ix_(xs, cols[:-1])])) ** 2 if xs else 1.0
    w = np.zeros(L)
    for y in range(L):
        if y in xs:
            continue
        w[y] = abs(np.linalg.det(U[np.ix_(xs + [y], cols)])) ** 2 / base
    return w


def inverse_cdf(w, u):
    """Draw by inverse CDF over ascending sites.

    F = running float64 sum of w (sequential), T = F[-1]; x = first site with
    F[x] > u*T.  Also returns T and the relative distance of u*T to the
    nearer end of x's interval (the near-tie margin used to classify any
    GPU/oracle disagreement).
    """
    F = np.cumsum(w)
    T = F[-1]
    if not (T > 0.0) or not np.isfinite(T):
        raise FloatingPointError("conditional weights have no mass (T=%r)" % T)
    target = u * T
    x = int(np.searchsorted(F, target, side="right"))
    if x >= len(w):
        raise FloatingPointError("inverse CDF ran off the end")
    lo = F[x - 1] if x > 0 else 0.0
    margin = min(target - lo, F[x] - target) / T
    return x, T, margin


def column_order(seed, sample, N, n_steps=None):
    """The first n_steps entries of the sample's column order m (0-based)."""
    n_steps = N if n_steps is None else n_steps
    perm = list(range(N))
    for t in range(n_steps):
        wds = philox.step_words(seed, sample, t)
        j = philox.fisher_yates_index(wds, t, N)
        perm[t], perm[j] = perm[j], perm[t]
    return perm[:n_steps]


def sample_one(U, seed, sample, n_keep=None):
    """One configuration (draw order) for (seed, sample): the FFS algorithm.

    Returns dict with x (list), logdet = sum_k log w_k(x_k) with w the
    unnormalised weight (= log|det U[x, m]|^2 when n_keep = N), and per-step
    margins and totals.
    """
    U = np.asarray(U)
    L, N = U.shape
    n_keep = N if n_keep is None else int(n_keep)
    perm = list(range(N))
    xs, margins, totals = [], [], []
    logdet = 0.0
    for t in range(n_keep):
        wds = philox.step_words(seed, sample, t)
        j = philox.fisher_yates_index(wds, t, N)
        perm[t], perm[j] = perm[j], perm[t]
        w = conditional_weights(U, xs, perm[: t + 1])
        x, T, margin = inverse_cdf(w, philox.uniform53(wds))
        logdet += float(np.log(w[x]))
        xs.append(x)
        margins.append(margin)
        totals.append(T)
    return {"x": xs, "logdet": logdet, "margin": margins, "T": totals,
            "m": perm[:n_keep]}


def sample(U, seed, first_sample, n_samples, n_keep=None):
    """Configurations for samples first_sample .. first_sample+n_samples-1.

    Returns (x int64 [n, n_keep], logdet float64 [n], min margin per sample).
    """
    N = np.asarray(U).shape[1]
    n_keep = N if n_keep is None else int(n_keep)
    X = np.zeros((n_samples, n_keep), dtype=np.int64)
    ld = np.zeros(n_samples)
    mm = np.ones(n_samples)
    for i in range(n_samples):
        r = sample_one(U, seed, first_sample + i, n_keep)
        X[i] = r["x"]
        ld[i] = r["logdet"]
        mm[i] = min(r["margin"]) if r["margin"] else 1.0
    return X, ld, mm


def teacher_forced_weights(U, seed, sample, prefix):
    """Normalised conditional at step k = len(prefix)+1 after a forced prefix.

    The column order is the sample's own (Philox stream of (seed, sample)).
    """
    U = np.asarray(U)
    N = U.shape[1]
    k = len(prefix) + 1
    cols = column_order(seed, sample, N, k)
    w = conditional_weights(U, list(prefix), cols)
    return w / np.cumsum(w)[-1]


def density(U):
    """One-particle density diag(U U^dagger): the site marginals, sum = N."""
    U = np.asarray(U)
    return _abs2(U).sum(axis=1)
