"""Metropolis conditional update, the large-L / continuous variant (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

SI S-7: the column order m is drawn as in the main algorithm; each x_k is then
drawn from its conditional P(x_k | x_<k; m) by a Markov chain on the single
variable x_k instead of the explicit all-site draw: a proposal x_k -> x' is
accepted with probability |u_{x'}^T h|^2 / |u_{x_k}^T h|^2 (capped at 1), h
the normal vector of Eq. (3), iterated M_cond times.  For a lattice the
continuous move x + dx becomes a discrete move x -> x'.

Readings of points the supplement leaves open (same on the GPU side):
  * the chain for x_k starts at the anchor of column m_k, the first row of
    largest |U[., m_k]|^2 (where the new orbital's weight concentrates);
    proposals are c + d with d uniform in [-R, -1] u [1, R] (modulo L) for a
    radius R > 0, or uniform over the L sites for R = 0; both are symmetric,
    so the acceptance ratio is the weight ratio;
  * iteration j of step t of a sample uses the Philox block keyed
    (seed, sample, step = t) with counter word 3 = 2 + j: the proposal from
    words 0,1 by 64-bit multiply-high, u = uniform53 from words 2,3;
    y is accepted when u * w(c) < w(y) (occupied sites weigh 0);
  * a chain that ends on a site of weight 0 (an occupied anchor, nothing
    accepted) moves to the nearest free site of positive weight, distance
    1, 2, ... from it, the lower side first.
"""
import numpy as np

from . import philox
from .sampler import _abs2, conditional_amplitudes

MH_STREAM0 = 2


def _mulhi(words, r):
    v = (words[1] << 32) | words[0]
    return (v * r) >> 64


def sample_one_mh(U, seed, sample, m_cond, radius=0, n_keep=None):
    """One configuration by the Metropolis conditional update.

    Returns dict with x, logdet (sum of log w(x_k)), accepted proposals, and
    per step the smallest relative gap |u w(c) - w(y)| / max(u w(c), w(y))
    of its acceptance tests (how near a float64 tie the chain came)."""
    U = np.asarray(U)
    L, N = U.shape
    n_keep = N if n_keep is None else int(n_keep)
    perm = list(range(N))
    anchor = [int(np.argmax(_abs2(U[:, c]))) for c in range(N)]
    xs = []
    logdet = 0.0
    accepted = 0
    gaps = []
    for t in range(n_keep):
        wds = philox.step_words(seed, sample, t)
        j = philox.fisher_yates_index(wds, t, N)
        perm[t], perm[j] = perm[j], perm[t]
        v, _ = conditional_amplitudes(U, xs, perm[: t + 1])
        w = _abs2(v)
        w[xs] = 0.0
        cur = anchor[perm[t]]
        wc = float(w[cur])
        gap = 1.0
        for it in range(m_cond):
            b = philox.stream_words(seed, sample, t, MH_STREAM0 + it)
            if radius == 0:
                y = _mulhi(b, L)
            else:
                r = _mulhi(b, 2 * radius)
                d = r - radius if r < radius else r - radius + 1
                y = (cur + d) % L
            u = philox.uniform53(b)
            big = max(u * wc, float(w[y]))
            if big > 0.0:
                gap = min(gap, abs(u * wc - float(w[y])) / big)
            if u * wc < w[y]:
                cur, wc = y, float(w[y])
                accepted += 1
        if not wc > 0.0:
            found = None
            for dist in range(1, L):
                for y in (cur - dist, cur + dist):
                    if 0 <= y < L and y not in xs and w[y] > 0.0:
                        found = y
                        break
                if found is not None:
                    break
            cur = found if found is not None else [y for y in range(L) if y not in xs][0]
        logdet += float(np.log(w[cur])) if w[cur] > 0 else -np.inf
        xs.append(cur)
        gaps.append(gap)
    return {"x": xs, "logdet": logdet, "accepted": accepted, "m": perm[:n_keep],
            "gap": gaps}
