"""Slater-Jastrow reweighting (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

SI S-5, Eq. (S8): for psi_J = J psi_0 with J diagonal in the position basis,
<O>_J = sum_x J^2(x) |psi_0(x)|^2 o_L(x) / sum_x J^2(x) |psi_0(x)|^2
      = <J^2 o_L>_0 / <J^2>_0,
so draws of the free-fermion ensemble |psi_0|^2 are reweighted by J^2.

Readings (same on the GPU side):
  * spin-1/2 fermions: a configuration is a pair (x_up, x_dn) of draws,
    |psi_0|^2 the product of the two determinant laws; -1 marks an empty
    slot of a row;
  * log J^2(x) = -V D(x) - sum_{i,j} v_ij n_i n_j (+ an optional per-sample
    log-weight): D = number of sites holding both spins (the main text's
    Gutzwiller factor J = exp(-V/2 sum_i n_i,up n_i,dn)), n_i = n_i,up +
    n_i,dn (the general density Jastrow of SI S-5);
  * observables are diagonal (site densities, D), so o_L(x) is their value;
  * weights w_s = exp(log J^2(x_s) - m), m = max_s log J^2(x_s) (the shift
    cancels in the ratio).
"""
import itertools

import numpy as np


def _sites(row):
    return [int(y) for y in row if int(y) >= 0]


def log_weights(x_up, x_dn, V, vmat=None, extra=None):
    """log J^2 of every sample (plus extra), and the double occupancies D."""
    n = len(x_up)
    lw = np.zeros(n)
    D = np.zeros(n, dtype=np.int64)
    for s in range(n):
        up = _sites(x_up[s])
        dn = _sites(x_dn[s]) if x_dn is not None else []
        D[s] = len(set(up) & set(dn))
        val = -V * D[s]
        if vmat is not None:
            occ = up + dn
            val -= sum(vmat[a, b] for a in occ for b in occ)
        if extra is not None:
            val += extra[s]
        lw[s] = val
    return lw, D


def estimate(x_up, x_dn, L, V, vmat=None, extra=None):
    """(logw, <n_i>_J for i < L, summary) with summary = (<D>_J, <D>_0,
    sum w, sum w^2, effective sample size, shift m)."""
    lw, D = log_weights(x_up, x_dn, V, vmat, extra)
    m = lw.max()
    w = np.exp(lw - m)
    dens = np.zeros(L)
    for s in range(len(x_up)):
        for y in _sites(x_up[s]):
            dens[y] += w[s]
        if x_dn is not None:
            for y in _sites(x_dn[s]):
                dens[y] += w[s]
    sw, sw2 = w.sum(), (w * w).sum()
    summary = (float((w * D).sum() / sw), float(D.mean()), float(sw), float(sw2),
               float(sw * sw / sw2), float(m))
    return lw, dens / sw, summary


def exact(U_up, U_dn, V, vmat=None):
    """<n_i>_J and <D>_J by enumerating every pair of site sets (tiny L)."""
    L, Nu = U_up.shape
    Nd = U_dn.shape[1]
    dens = np.zeros(L)
    Dm = 0.0
    Z = 0.0
    for xu in itertools.combinations(range(L), Nu):
        pu = abs(np.linalg.det(U_up[list(xu)])) ** 2
        for xd in itertools.combinations(range(L), Nd):
            pd = abs(np.linalg.det(U_dn[list(xd)])) ** 2
            D = len(set(xu) & set(xd))
            lj = -V * D
            if vmat is not None:
                occ = list(xu) + list(xd)
                lj -= sum(vmat[a, b] for a in occ for b in occ)
            wt = pu * pd * np.exp(lj)
            Z += wt
            Dm += wt * D
            for y in xu:
                dens[y] += wt
            for y in xd:
                dens[y] += wt
    return dens / Z, Dm / Z
