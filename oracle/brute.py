"""Brute-force optimal assignment by enumeration of all permutations (n <= 8).

Test infrastructure: the plain definition of the optimal assignment problem,
max over permutations sigma of sum_i b_{i sigma(i)} (Section 2.2), used to pin
the oracle's Hungarian solver and the certificate.
"""
from __future__ import annotations

import itertools
import math


def all_optima(b, tol=0.0):
    """Returns (best value, list of optimal permutations) for a square matrix
    b (nested lists or an array) of log-weights; -inf entries are forbidden."""
    n = len(b)
    assert n <= 8, "brute force is for n <= 8"
    best = -math.inf
    winners = []
    for perm in itertools.permutations(range(n)):
        s = 0.0
        for i in range(n):
            s += float(b[i][perm[i]])
        if s == -math.inf:
            continue
        if s > best + tol:
            best = s
            winners = [perm]
        elif abs(s - best) <= tol:
            winners.append(perm)
    return best, winners


def permutation_weights(b):
    """Dictionary perm -> sum_i b_{i perm(i)} over all permutations."""
    n = len(b)
    assert n <= 8
    return {perm: sum(float(b[i][perm[i]]) for i in range(n))
            for perm in itertools.permutations(range(n))}
