"""GPU parity cases for paths the standard workloads rarely or never reach.

  * High degrees (16..63), explicit edge lists: with 5 to 8 chains per unit
    the 4-bit unsatisfied-bond counts would overflow, so those chunks take the
    8-bit even/odd count path; with 1, 2 or 4 chains the wider fields count
    directly and neighbours beyond the prefetched eight are re-read.  Each
    packing runs on a graph whose adjacency is LDS-resident and on one that
    is streamed from HBM.
  * Long runs: 2^17 sweeps over many calls of uneven length (sweep counters
    above 2^12, grid indices up to 17, launch lengths at their cap).
  * Instances that pass the same edge arrays with different seeds (separate
    units).
  * The SK integrity check: a local field corrupted between sweeps is
    reported by the next exact recomputation.

Everything is compared with the oracle element by element (all integers)."""
import concurrent.futures as cf
import math

import numpy as np
import pytest

import paper_1906_11195_amd as sg
from tests.gpu_util import assert_instance_equal, oracle_sk, oracle_vb, require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS
HUB_DEGREES = (16, 17, 19, 24, 31, 32, 33, 40, 47, 48, 55, 63)


def hub_graph(n, c, seed, hubs=HUB_DEGREES):
    """A sparse random graph (about c n / 2 edges) plus hub vertices with the
    given degrees, as an explicit edge list with +-1 couplings: simple, and
    no degree above 63.  Hubs sit in different colour classes and chunks."""
    rng = np.random.default_rng(seed)
    edges = set()
    deg = np.zeros(n, np.int64)

    def add(u, v):
        if u == v:
            return False
        key = (min(u, v), max(u, v))
        if key in edges or deg[u] >= 63 or deg[v] >= 63:
            return False
        edges.add(key)
        deg[u] += 1
        deg[v] += 1
        return True

    m = int(c * n / 2)
    while len(edges) < m:
        u, v = rng.integers(0, n, size=2)
        add(int(u), int(v))
    hub_ids = rng.choice(n, size=len(hubs), replace=False)
    is_hub = np.zeros(n, bool)
    is_hub[hub_ids] = True
    for h, want in zip(hub_ids, hubs):
        h = int(h)
        while deg[h] < want:
            v = int(rng.integers(0, n))
            if not is_hub[v]:
                add(h, v)
    e = np.array(sorted(edges), np.int32)
    e = e[rng.permutation(len(e))]
    J = rng.choice([-1, 1], size=len(e)).astype(np.int8)
    assert deg.max() <= 63 and set(int(x) for x in deg[hub_ids]) == set(hubs)
    return e, J


def run_lib(descs, chunks, t_max, **kw):
    ctx = sg.sg_create_vb(descs, t_max=t_max, **kw)
    try:
        for k in chunks:
            sg.sg_sweep(ctx, k)
        return sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)


def oracle_all(descs, n_sweeps, t_max):
    with cf.ThreadPoolExecutor(max_workers=min(16, len(descs))) as ex:
        return list(ex.map(lambda d: oracle_vb(d, n_sweeps, t_max), descs))


# (chains per unit, instances, replicas): 8, 7, 6, 5 chains take the 8-slot
# units (4-bit fields, 8-bit path for chunks with a degree above 15); 4, 2, 1
# chains the 4, 2 and 1-slot units
PACKINGS = [(8, 4, 2), (7, 7, 1), (6, 3, 2), (5, 5, 1), (4, 2, 2), (2, 1, 2), (1, 1, 1)]


# plain_lds: units that stream their adjacency keep no complemented copy of
# the spin words (the sign of J is applied to the word read) instead of
# addressing the copy
@pytest.mark.parametrize("plain_lds", [False, True])
@pytest.mark.parametrize("n", [3001, 40007])
@pytest.mark.parametrize("cpu,n_inst,R", PACKINGS)
def test_vb_high_degree_every_packing(n, cpu, n_inst, R, plain_lds):
    require_gpu()
    e, J = hub_graph(n, 4.0, seed=n)
    temps = [0.9, 3.0, math.inf, 1.6, 0.5, 2.2, 0.0][:n_inst]
    descs = [sg.VbDesc(n=n, T=T, seed=21, instance_id=40 + k, edges=e, J=J, n_replicas=R)
             for k, T in enumerate(temps)]
    res = run_lib(descs, [17, 23], 32, chains_per_unit=cpu, plain_lds=plain_lds)
    for i, ref in enumerate(oracle_all(descs, 40, 32)):
        assert_instance_equal(res, i, ref, label="n=%d cpu=%d inst %d" % (n, cpu, i))


def test_vb_long_run_over_many_calls():
    # 3 temperatures x 2 replicas on one graph (a 6-chain unit), 2^17 + 3
    # sweeps in calls of uneven length, compared at every grid time
    require_gpu()
    n = 384
    total = (1 << 17) + 3
    descs = [sg.VbDesc(n=n, T=T, seed=9, instance_id=k, graph_id=4, c=4.0)
             for k, T in enumerate([0.6, 0.8, 1.2])]
    chunks, left, step = [], total, 1
    while left > 0:
        k = min(left, step)
        chunks.append(k)
        left -= k
        step = step * 3 + 7 if step < 9000 else 4093
    res = run_lib(descs, chunks, 1 << 17)
    assert res["t_done"] == total and res["k_done"] == 19
    for i, ref in enumerate(oracle_all(descs, total, 1 << 17)):
        assert_instance_equal(res, i, ref, label="long inst %d" % i)
        assert ref["accepted"].min() > (1 << 20)


def test_vb_shared_arrays_mixed_seeds():
    # the same edge arrays with two seeds: separate units (each unit's chains
    # share one Philox key); both equal the oracle and the runs alone
    require_gpu()
    n = 5000
    e, J = hub_graph(n, 4.0, seed=3, hubs=(20,))
    descs = [sg.VbDesc(n=n, T=T, seed=seed, instance_id=k, edges=e, J=J)
             for k, (T, seed) in enumerate([(0.8, 1), (0.8, 2), (1.1, 1), (1.1, 7)])]
    res = run_lib(descs, [50], 64)
    refs = oracle_all(descs, 50, 64)
    for i, ref in enumerate(refs):
        assert_instance_equal(res, i, ref, label="seed mix inst %d" % i)
    alone = run_lib(descs[1:2], [50], 64)
    assert_instance_equal(alone, 0, refs[1], label="alone")


def test_sk_corrupted_field_is_reported_by_the_recompute():
    # A field corrupted from the host between sweeps is caught at the next
    # exact recomputation (every 64 sweeps), not before; an intact context of
    # the same instance stays equal to the oracle.
    require_gpu()
    n = 300
    d = sg.SkDesc(n=n, T=0.5, seed=3, instance_id=2, graph_id=1, recompute_period=64)
    ctx = sg.sg_create_sk([d], t_max=256)
    try:
        sg.sg_sweep(ctx, 64)
        ok = sg.sg_measure(ctx, FLAGS)
        assert_instance_equal(ok, 0, oracle_sk(d, 64, 256), label="before")
        sg.sg_sk_corrupt_field(ctx, 0, 1, 123, 2)
        sg.sg_sweep(ctx, 63)
        assert sg.sg_measure(ctx, FLAGS, check=False)["status"] == sg.SG_OK
        sg.sg_sweep(ctx, 1)
        assert sg.sg_measure(ctx, FLAGS, check=False)["status"] == sg.SG_EPARITY
        sg.sg_sweep(ctx, 64)
        assert sg.sg_measure(ctx, FLAGS, check=False)["status"] == sg.SG_EPARITY
        with pytest.raises(sg.SgError):
            sg.sg_sk_corrupt_field(ctx, 1, 0, 0, 1)
    finally:
        sg.sg_free(ctx)
    ctx = sg.sg_create_sk([d], t_max=256)
    try:
        sg.sg_sweep(ctx, 192)
        assert_instance_equal(sg.sg_measure(ctx, FLAGS), 0, oracle_sk(d, 192, 256), label="intact")
    finally:
        sg.sg_free(ctx)
