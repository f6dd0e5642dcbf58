"""GPU parity of the multispin layout (SG_OPT_MULTISPIN: up to 64 chains of
one graph per 64-bit word, each chain with its own couplings, temperature
and random streams).  Every chain's observables and final spins equal the
oracle's for its own coupling array, and equal the per-chain layout's,
element by element (all integers): partial units, several units of one
graph, replicas, degrees above 15 (the wide counter), aligned and given
starts, sweeps over several calls, graph replay, and multispin units next to
per-chain ones in one context."""
import concurrent.futures as cf
import math

import numpy as np
import pytest

import oracle
import paper_1906_11195_amd as sg
from paper_1906_11195_amd.workloads import random_regular_edges
from tests.gpu_util import assert_instance_equal, oracle_vb, require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS


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


def samples_on(edges, n_inst, n, T, seed, R=1, inst0=0, **kw):
    """n_inst instances on one edge array, each with its own +-1 couplings."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        J = rng.choice([-1, 1], size=len(edges)).astype(np.int8)
        TT = T[k % len(T)] if isinstance(T, (list, tuple)) else T
        out.append(sg.VbDesc(n=n, T=TT, seed=seed, instance_id=inst0 + k, edges=edges, J=J, n_replicas=R, **kw))
    return out


def check(descs, chunks, t_max, **kw):
    ms = run_lib(descs, chunks, t_max, multispin=True, **kw)
    pc = run_lib(descs, chunks, t_max, multispin=False, **kw)
    refs = oracle_all(descs, sum(chunks), t_max)
    for i, ref in enumerate(refs):
        assert_instance_equal(ms, i, ref, label="multispin inst %d" % i)
        assert_instance_equal(pc, i, ref, label="per-chain inst %d" % i)


def test_multispin_rrbg_full_and_partial_units():
    require_gpu()
    n = 2000
    e, _ = random_regular_edges(n, 4, seed=5, bipartite=True)
    # 100 samples: one full unit of 64 and one of 36
    descs = samples_on(e, 100, n, [0.6, 0.9, 1.3, math.inf, 0.0], seed=3)
    check(descs, [37, 27], 64)


def test_multispin_replicas_er_degrees_and_starts():
    require_gpu()
    n = 3001
    rng = np.random.default_rng(8)
    # an ER-like graph with degrees up to ~20 (the wide counter) as explicit edges
    pairs = set()
    while len(pairs) < 2 * n:
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u != v:
            pairs.add((min(u, v), max(u, v)))
    hub = 17
    for v in range(1, 23):
        if v != hub:
            pairs.add((min(hub, v), max(hub, v)))
    e = np.array(sorted(pairs), np.int32)
    s0 = rng.choice([-1, 1], size=(2, n)).astype(np.int8)
    descs = samples_on(e, 12, n, [0.8, 1.1], seed=9, R=2)
    descs[3].start = sg.START_ALIGNED
    descs[5].start = sg.START_GIVEN
    descs[5].s0 = s0
    check(descs, [1, 20, 43], 64)


def test_multispin_next_to_per_chain_units_and_graph_replay():
    require_gpu()
    n = 1500
    e, _ = random_regular_edges(n, 4, seed=11, bipartite=False)
    many = samples_on(e, 40, n, 0.7, seed=4)                       # multispin (40 chains)
    few = [sg.VbDesc(n=777, T=0.9, seed=4, instance_id=100 + k, graph_id=k, n_replicas=1)
           for k in range(3)]                                          # per-chain (one replica, as above)
    descs = many + few
    check(descs, [50, 14], 64, graph=True)


def test_multispin_generated_graph_shares_couplings():
    require_gpu()
    # 9 instances x 2 replicas on one generated graph: 18 chains, one unit
    descs = [sg.VbDesc(n=4096, T=T, seed=2, instance_id=k, graph_id=1) for k, T in
             enumerate([0.6, 0.8, 1.2] * 3)]
    check(descs, [64], 64)


def test_multispin_benchmark_shape_sampled():
    # units of the benchmark's multispin leg (RRBG, N = 8192, 32 coupling
    # samples x 2 replicas per graph): four graphs, a prefix of 24 sweeps,
    # sampled instances against the oracle
    require_gpu()
    from paper_1906_11195_amd import workloads
    descs = workloads.vb_multispin_batched(n_graphs=4)
    res = run_lib(descs, [10, 14], workloads.VB_BATCHED_SWEEPS, multispin=True)
    picks = [0, 31, 45, 127]
    refs = oracle_all([descs[i] for i in picks], 24, workloads.VB_BATCHED_SWEEPS)
    for i, ref in zip(picks, refs):
        assert_instance_equal(res, i, ref, label="bench-shape inst %d" % i)
