"""Brute-force enumerators for tiny systems (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

These compute, by exhaustive enumeration, (a) the target law of Eq. (1) over
ordered configurations and (b) the exact law of the FFS sampler: the average
over all N! column orders m of the product of normalised conditionals
(Eq. (2)).  Eq. (2) says the two coincide; the tests check that numerically.
"""
import itertools
import math

import numpy as np

from . import sampler


def det_law(U):
    """{ordered x: |det U[x,:]|^2 / N!} over all ordered N-tuples (Eq. (1))."""
    U = np.asarray(U)
    L, N = U.shape
    f = math.factorial(N)
    return {x: abs(np.linalg.det(U[list(x), :])) ** 2 / f
            for x in itertools.permutations(range(L), N)}


def sampler_law(U, weight_fn=None):
    """Exact law of the sampler: (1/N!) sum_m prod_k w_k(x_k | x_<k; m)."""
    U = np.asarray(U)
    L, N = U.shape
    weight_fn = sampler.conditional_weights if weight_fn is None else weight_fn
    law = {}
    pm = 1.0 / math.factorial(N)

    def rec(m, xs, p):
        k = len(xs)
        if k == N:
            law[tuple(xs)] = law.get(tuple(xs), 0.0) + p
            return
        w = weight_fn(U, xs, list(m[: k + 1]))
        w = w / w.sum()
        for y in range(L):
            if w[y] > 0.0:
                rec(m, xs + [y], p * w[y])

    for m in itertools.permutations(range(N)):
        rec(m, [], pm)
    return law


def set_law(ordered_law):
    """Collapse an ordered law onto unordered sets (sorted tuples)."""
    out = {}
    for x, p in ordered_law.items():
        key = tuple(sorted(x))
        out[key] = out.get(key, 0.0) + p
    return out


def cauchy_binet_total(U):
    """sum over N-subsets S of |det U[S,:]|^2; equals det(U^dagger U) = 1."""
    U = np.asarray(U)
    L, N = U.shape
    return sum(abs(np.linalg.det(U[list(S), :])) ** 2
               for S in itertools.combinations(range(L), N))
