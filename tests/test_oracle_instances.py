"""Pins for the oracle's instance builders: ER graph, SK couplings, greedy
colouring, sweep order and Metropolis threshold tables (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from tests import brute


def test_er_graph_is_simple_with_m_edges():
    n, c = 4096, 4.0
    m = oracle.n_edges(n, c)
    assert m == 8192
    eu, ev, J, attempts = oracle.er_graph(n, m, seed=2, graph_id=7)
    assert len(eu) == m and attempts >= m
    assert np.all(eu != ev)
    assert eu.min() >= 0 and ev.max() < n and eu.max() < n and ev.min() >= 0
    pairs = set(zip(np.minimum(eu, ev).tolist(), np.maximum(eu, ev).tolist()))
    assert len(pairs) == m
    assert set(np.unique(J)) == {-1, 1}


def test_er_graph_deterministic_and_keyed():
    a = oracle.er_graph(1024, 2048, 1, 0)
    b = oracle.er_graph(1024, 2048, 1, 0)
    c = oracle.er_graph(1024, 2048, 1, 1)
    d = oracle.er_graph(1024, 2048, 2, 0)
    assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3]))
    assert not np.array_equal(a[0], c[0])
    assert not np.array_equal(a[0], d[0])


def test_er_degree_distribution_is_poisson_and_couplings_balanced():
    n, c = 65536, 4.0
    m = oracle.n_edges(n, c)
    eu, ev, J, _ = oracle.er_graph(n, m, seed=9, graph_id=0)
    deg = np.bincount(np.concatenate([eu, ev]), minlength=n)
    assert deg.sum() == 2 * m
    # G(N, M) degrees are Binomial(N-1, 2M/(N(N-1))) ~ Poisson(c) at this size.
    kmax = 12
    obs = np.array([np.sum(deg == k) for k in range(kmax)] + [np.sum(deg >= kmax)], float)
    p = np.array([stats.poisson.pmf(k, c) for k in range(kmax)] + [stats.poisson.sf(kmax - 1, c)])
    chi2, pval = stats.chisquare(obs, p * n)
    assert pval > 1e-4
    # +-1 couplings with probability 1/2 each
    assert stats.binomtest(int(np.sum(J == 1)), m, 0.5).pvalue > 1e-4
    # endpoint uniformity
    hist = np.bincount(np.concatenate([eu, ev]) * 16 // n, minlength=16)
    assert stats.chisquare(hist).pvalue > 1e-4


def test_greedy_colouring_proper_and_greedy():
    n = 2000
    eu, ev, J, _ = oracle.er_graph(n, oracle.n_edges(n, 4.0), seed=5, graph_id=1)
    colour, ncol = oracle.greedy_colour(n, eu, ev)
    assert np.all(colour[eu] != colour[ev])                     # proper
    deg = np.bincount(np.concatenate([eu, ev]), minlength=n)
    assert ncol == colour.max() + 1 <= deg.max() + 1
    # independent re-implementation on the same graph
    nbrs = [[] for _ in range(n)]
    for u, v in zip(eu.tolist(), ev.tolist()):
        nbrs[u].append(v)
        nbrs[v].append(u)
    ref = [-1] * n
    for v in range(n):
        taken = {ref[u] for u in nbrs[v] if u < v}
        k = 0
        while k in taken:
            k += 1
        ref[v] = k
    assert list(colour) == ref


def test_sweep_order_groups_classes_by_decreasing_degree():
    n = 3000
    eu, ev, J, _ = oracle.er_graph(n, oracle.n_edges(n, 4.0), seed=5, graph_id=2)
    colour, ncol = oracle.greedy_colour(n, eu, ev)
    deg = np.bincount(np.concatenate([eu, ev]), minlength=n)
    order = oracle.sweep_order(colour, ncol, deg)
    assert sorted(order.tolist()) == list(range(n))
    assert order.tolist() == sorted(range(n), key=lambda v: (colour[v], -deg[v], v))
    cs = colour[order]
    assert np.all(np.diff(cs) >= 0)
    for k in range(ncol):
        d = deg[order[cs == k]]
        assert np.all(np.diff(d) <= 0)


def test_sk_couplings_symmetric_balanced_zero_diagonal():
    n = 512
    J = oracle.sk_couplings(n, seed=3, graph_id=4)
    assert np.array_equal(J, J.T)
    assert np.all(np.diag(J) == 0)
    off = J[np.triu_indices(n, 1)]
    assert set(np.unique(off)) == {-1, 1}
    assert stats.binomtest(int(np.sum(off == 1)), len(off), 0.5).pvalue > 1e-4
    J2 = oracle.sk_couplings(n, seed=3, graph_id=5)
    assert not np.array_equal(J, J2)
    # the same (seed, graph_id) at another size is a different matrix (idx = i*N + j)
    assert not np.array_equal(oracle.sk_couplings(256, 3, 4), J[:256, :256])


@pytest.mark.parametrize("T", [0.5, 0.8, 1.2, 3.0])
def test_thresholds_match_metropolis_closed_form(T):
    thr = oracle.thresholds(T, 1.0, 16)
    assert thr[0] == 2**32
    for x in range(1, 17):
        p = math.exp(-2.0 * x / T)                 # min(1, e^{-beta dE}), dE = 2x
        assert abs(int(thr[x]) / 2**32 - p) <= 2.0**-32
        assert int(thr[x]) <= p * 2**32 < int(thr[x]) + 1
    assert np.all(np.diff(thr.astype(np.float64)) <= 0)


def test_thresholds_limits_and_sk_scale():
    inf = oracle.thresholds(math.inf, 1.0, 8)
    assert np.all(inf == 2**32)                    # T = inf: every move accepted
    zero = oracle.thresholds(0.0, 1.0, 8)
    assert zero[0] == 2**32 and np.all(zero[1:] == 0)   # T = 0: only x <= 0 moves
    n = 4096
    sk = oracle.thresholds(0.5, 1.0 / math.sqrt(n), n - 1)
    for x in (1, 2, 10, 100, 354):
        p = math.exp(-2.0 * (2.0 * x / math.sqrt(n)))
        assert abs(int(sk[x]) / 2**32 - p) <= 2.0**-32
    assert sk[355] == 0 and sk[354] > 0


def test_grid():
    assert oracle.grid(4096).tolist() == [0] + [2**k for k in range(13)]
    assert oracle.grid(0).tolist() == [0]
    assert oracle.grid(5).tolist() == [0, 1, 2, 4]
    assert len(oracle.grid(2**20)) == 22
