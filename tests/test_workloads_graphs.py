"""The random regular (bipartite) graph inputs: every vertex has degree z, the
graph is simple, the bipartite one only joins the two halves, and a seed
fixes the graph."""
import numpy as np
import pytest

from paper_1906_11195_amd import workloads as W


def _check(n, z, e, J, bipartite):
    assert e.shape == (n * z // 2, 2) and e.dtype == np.int32
    assert J.shape == (n * z // 2,) and set(np.unique(J).tolist()) <= {-1, 1}
    assert np.array_equal(np.bincount(e.ravel(), minlength=n), np.full(n, z))
    assert not np.any(e[:, 0] == e[:, 1])
    codes = np.minimum(e[:, 0], e[:, 1]).astype(np.int64) * n + np.maximum(e[:, 0], e[:, 1])
    assert len(np.unique(codes)) == len(codes)
    if bipartite:
        assert np.all(e[:, 0] < n // 2) and np.all(e[:, 1] >= n // 2)


@pytest.mark.parametrize("n,z,bipartite", [(16, 4, False), (16, 4, True), (1000, 4, False), (4096, 4, True),
                                           (65536, 4, True), (2001, 6, False)])
def test_random_regular_graphs_are_simple_and_regular(n, z, bipartite):
    e, J = W.random_regular_edges(n, z, seed=11 + n, bipartite=bipartite)
    _check(n, z, e, J, bipartite)


def test_random_regular_graph_is_fixed_by_its_seed():
    a = W.random_regular_edges(4096, 4, seed=3, bipartite=True)
    b = W.random_regular_edges(4096, 4, seed=3, bipartite=True)
    c = W.random_regular_edges(4096, 4, seed=4, bipartite=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])


def test_rrbg_recipe_shares_arrays_between_temperatures():
    descs = W.vb_rrbg_batched(n_graphs=2, n=1024)
    assert len(descs) == 6
    assert descs[0].edges is descs[1].edges is descs[2].edges and descs[0].J is descs[2].J
    assert descs[3].edges is not descs[0].edges


@pytest.mark.parametrize("n,z,bipartite", [(4, 4, False), (8, 5, True), (7, 3, False), (7, 2, True)])
def test_impossible_regular_graphs_are_refused(n, z, bipartite):
    with pytest.raises(ValueError):
        W.random_regular_edges(n, z, seed=1, bipartite=bipartite)


def test_dense_regular_graph_is_found():
    # the complete graph K5 is the only 4-regular simple graph on 5 vertices
    e, J = W.random_regular_edges(5, 4, seed=2)
    _check(5, 4, e, J, False)
