"""DPP front end (oracle side): dual eigendecomposition, eigenvector selection.

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

The paper's subset-selection application (applications section, text
summarisation): items i carry vectors b_i (the rows of B, quality folded into
their norms), the DPP kernel is C = B B^T, and a draw keeps each eigenvector
u_j of C with probability lambda_j / (lambda_j + 1), then samples the items
as fermions in the kept eigenvectors (Eq. (1) with U = the kept columns).
The fixed-size variant (a k-DPP) keeps a k-subset J with probability
prod_{j in J} lambda_j / e_k(lambda) (Kulesza and Taskar's review of DPPs,
elementary symmetric polynomial selection).

Readings of points the paper leaves open (same on the GPU side):
  * the nonzero spectrum of C is taken through the dual B^T B: if
    B^T B w = lambda w then u = B w / sqrt(lambda) is a unit eigenvector of
    C with the same eigenvalue;
  * eigenvalues ascending; each w_j signed so that its largest-magnitude
    entry (the first one on ties) is positive;
  * the selection uniforms are Philox blocks keyed (seed, sample, step = j)
    with counter word 3 = 1, u = uniform53 (philox.py);
  * k-DPP: mu = lambda / max(lambda) (the selection rule does not depend on
    the scale; this one keeps e_m in range), E[m][j] = e_m(mu_0..mu_{j-1})
    by E[m][j] = E[m][j-1] + mu_{j-1} E[m-1][j-1]; j runs from d-1 down and,
    with l indices left, j is kept when j + 1 == l or
    u_j < (mu_j E[l-1][j]) / E[l][j+1].  Products and sums are rounded one
    at a time (no fused multiply-add), in this order.
"""
import numpy as np

from . import philox

SELECT_STREAM = 1


def dual_eig(B):
    """Eigenpairs of C = B B^T via B^T B: (lam ascending, U = B W / sqrt(lam), W)."""
    B = np.asarray(B, dtype=np.float64)
    lam, W = np.linalg.eigh(B.T @ B)
    for j in range(W.shape[1]):
        r = int(np.argmax(np.abs(W[:, j])))  # first maximum
        if W[r, j] < 0.0:
            W[:, j] = -W[:, j]
    U = (B @ W) / np.sqrt(lam)[None, :]
    return lam, U, W


def esp_table(lam, k):
    """E[m][j] = e_m(mu_0..mu_{j-1}), mu = lam / max(lam); shape (k+1, d+1)."""
    lam = [float(v) for v in lam]
    d = len(lam)
    top = max(lam)
    mu = [v / top for v in lam]
    E = [[0.0] * (d + 1) for _ in range(k + 1)]
    E[0] = [1.0] * (d + 1)
    for m in range(1, k + 1):
        for j in range(1, d + 1):
            prod = mu[j - 1] * E[m - 1][j - 1]
            E[m][j] = E[m][j - 1] + prod
    return np.array(E)


def kdpp_select(lam, k, seed, sample, E=None):
    """Sorted k-subset of eigenvector indices for one sample (k-DPP)."""
    lam = [float(v) for v in lam]
    d = len(lam)
    if E is None:
        E = esp_table(lam, k)
    top = max(lam)
    keep = []
    left = k
    for j in range(d - 1, -1, -1):
        if left == 0:
            break
        u = philox.uniform53(philox.stream_words(seed, sample, j, SELECT_STREAM))
        mu = lam[j] / top
        p = (mu * float(E[left - 1][j])) / float(E[left][j + 1])
        if j + 1 == left or u < p:
            keep.append(j)
            left -= 1
    return sorted(keep)


def dpp_select(lam, seed, sample):
    """Eigenvector indices kept by the DPP rule u_j < lam_j / (lam_j + 1)."""
    keep = []
    for j, v in enumerate(lam):
        v = float(v)
        u = philox.uniform53(philox.stream_words(seed, sample, j, SELECT_STREAM))
        if u < v / (v + 1.0):
            keep.append(j)
    return keep
