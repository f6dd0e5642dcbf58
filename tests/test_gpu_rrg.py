"""GPU parity on the paper's graph ensemble: random regular graphs of degree 4
and random regular bipartite graphs (explicit edge lists).  Instances that pass
the same arrays share one graph in a work unit; sharing changes no result."""
import numpy as np
import pytest

import paper_1906_11195_amd as sg
from paper_1906_11195_amd import workloads as W
from tests.gpu_util import assert_instance_equal, oracle_vb, require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS


def run_lib(descs, chunks, t_max):
    ctx = sg.sg_create_vb(descs, t_max=t_max)
    try:
        for k in chunks:
            sg.sg_sweep(ctx, k)
        return sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)


@pytest.mark.parametrize("n,bipartite", [(3001 * 2, False), (4096, True)])
def test_regular_graphs_match_oracle_shared_and_separate(n, bipartite):
    require_gpu()
    edges, J = W.random_regular_edges(n, 4, seed=17, bipartite=bipartite)
    temps = (0.6, 0.8, 1.2)
    shared = [sg.VbDesc(n=n, T=T, seed=6, instance_id=k, edges=edges, J=J) for k, T in enumerate(temps)]
    separate = [sg.VbDesc(n=n, T=T, seed=6, instance_id=k, edges=edges.copy(), J=J.copy())
                for k, T in enumerate(temps)]
    chunks = [3, 9]
    a = run_lib(shared, chunks, 16)
    b = run_lib(separate, chunks, 16)
    for key in ("bond", "overlap", "gram", "accepted"):
        assert np.array_equal(a[key], b[key]), key
    for i, d in enumerate(shared):
        assert_instance_equal(a, i, oracle_vb(d, sum(chunks), 16), label="rrg n=%d i=%d" % (n, i))
