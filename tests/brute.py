"""Brute-force references for tiny systems, written independently of the oracle.

Used only by the tests to pin the oracle.  Nothing here calls the oracle: the
colouring, the sweep order and the acceptance probabilities are recomputed in
plain numpy / Python from their definitions, and the acceptance probability is
the closed form min(1, exp(-beta dE)) in float64, not the oracle's quantised
threshold table (the two differ by less than 2^-32 per move).

States of N Ising spins are indexed by an integer whose bit i is 1 when
s_i = -1.
"""
from __future__ import annotations

import math

import numpy as np


def states(n: int) -> np.ndarray:
    idx = np.arange(1 << n, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1
    return (1 - 2 * bits).astype(np.int64)          # [2^n, n] of +-1


def coupling_matrix(n: int, eu, ev, J) -> np.ndarray:
    A = np.zeros((n, n), dtype=np.int64)
    for u, v, j in zip(eu, ev, J):
        A[u, v] += int(j)
        A[v, u] += int(j)
    return A


def bond_sum(S: np.ndarray, A: np.ndarray) -> np.ndarray:
    """B(s) = sum_{i<j} A_ij s_i s_j for every row of S."""
    return np.einsum("si,ij,sj->s", S, A, S) // 2


def greedy_colour(n: int, A: np.ndarray):
    colour = [-1] * n
    for v in range(n):
        taken = {colour[u] for u in range(v) if A[v, u] != 0}
        c = 0
        while c in taken:
            c += 1
        colour[v] = c
    return colour


def sweep_order(colour, A):
    """Colour classes in order; inside a class by decreasing degree, then id."""
    n = len(colour)
    deg = [int(np.count_nonzero(A[v])) for v in range(n)]
    return sorted(range(n), key=lambda v: (colour[v], -deg[v], v))


def accept_prob(x: np.ndarray, T: float, de_scale: float) -> np.ndarray:
    """min(1, exp(-beta * 2 x * de_scale)) with x = s_i h_i."""
    beta = 0.0 if math.isinf(T) else (math.inf if T == 0 else 1.0 / T)
    with np.errstate(over="ignore", invalid="ignore"):
        p = np.exp(-beta * 2.0 * x * de_scale) if beta != math.inf else np.zeros_like(x, float)
    return np.where(x <= 0, 1.0, p)


def site_update(dist: np.ndarray, S: np.ndarray, A: np.ndarray, v: int, T: float,
                de_scale: float) -> np.ndarray:
    """One Metropolis update of spin v applied to a distribution over states."""
    h = S @ A[v]                      # local field of v in every state
    x = S[:, v] * h
    a = accept_prob(x.astype(float), T, de_scale)
    partner = np.arange(len(dist)) ^ (1 << v)
    return dist * (1.0 - a) + dist[partner] * a[partner]


def sweep(dist, S, A, order, T, de_scale=1.0):
    for v in order:
        dist = site_update(dist, S, A, v, T, de_scale)
    return dist


def boltzmann(S, A, T, de_scale=1.0) -> np.ndarray:
    B = bond_sum(S, A).astype(float)
    w = np.exp((B - B.max()) * de_scale / T)
    return w / w.sum()
