"""GPU parity of VB units split over several workgroups (members that meet at a
device-scope barrier after every colour class and exchange the class's spin
words through HBM).  Splitting changes no result: every case is compared with
the oracle and with the same run unsplit, element by element."""
import numpy as np
import pytest

import paper_1906_11195_amd as sg
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


def assert_same(a, b, label):
    for key in ("bond", "overlap", "gram", "accepted"):
        assert np.array_equal(a[key], b[key]), (label, key)
    assert len(a["spins"]) == len(b["spins"])
    for i, (x, y) in enumerate(zip(a["spins"], b["spins"])):
        assert np.array_equal(x, y), (label, "spins", i)


@pytest.mark.parametrize("members,threads,rpad_chains", [(2, 64, 2), (3, 64, 1), (4, 128, 6), (5, 64, 4)])
def test_forced_split_matches_oracle(members, threads, rpad_chains):
    # one graph with 1, 2, 4 or 6 chains (3 temperatures x 2 replicas for 6),
    # ragged N, several launches (the barrier words are reset between them)
    require_gpu()
    n = 20011
    temps = [0.7, 1.1, 0.5][: max(1, rpad_chains // 2)]
    reps = 1 if rpad_chains == 1 else 2
    descs = [sg.VbDesc(n=n, T=T, seed=21, instance_id=10 + k, graph_id=3, c=4.0, n_replicas=reps)
             for k, T in enumerate(temps)]
    chunks = [5, 1, 26]
    res = run_lib(descs, chunks, 32, threads_per_unit=threads, split_members=members)
    ref_alone = run_lib(descs, chunks, 32, threads_per_unit=threads, split_members=1)
    assert_same(res, ref_alone, "split %d vs unsplit" % members)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_vb(d, sum(chunks), 32), label="members=%d i=%d" % (members, i))


def test_split_units_next_to_unsplit_ones_with_graph_replay():
    # a large graph split, small ones (LDS-resident adjacency) not; chunks
    # replayed from a captured graph, interleaved with plain launches
    require_gpu()
    descs = [sg.VbDesc(n=30000, T=0.8, seed=4, instance_id=0, graph_id=0, c=4.0)]
    descs += [sg.VbDesc(n=300 + 97 * k, T=0.6, seed=4, instance_id=1 + k, graph_id=1 + k, c=4.0)
              for k in range(5)]
    chunks = [8, 8, 3, 8]
    res = run_lib(descs, chunks, 16, threads_per_unit=64, split_members=4, graph=True)
    ref = run_lib(descs, chunks, 16, threads_per_unit=64, split_members=1)
    assert_same(res, ref, "graph + split vs plain")
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_vb(d, sum(chunks), 16), label="mixed i=%d" % i)


def test_automatic_split_of_one_large_graph():
    # one graph far above a CU's share of the batch is split automatically
    # (no option), and the result is still the oracle's
    require_gpu()
    descs = [sg.VbDesc(n=65536, T=0.9, seed=6, instance_id=0, graph_id=0, c=4.0)]
    descs += [sg.VbDesc(n=1024, T=0.9, seed=6, instance_id=1 + k, graph_id=1 + k, c=4.0) for k in range(3)]
    res = run_lib(descs, [6, 6], 8)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_vb(d, 12, 8), label="auto i=%d" % i)


def test_automatic_split_of_several_equal_graphs():
    # equal graphs far above a CU's share are all split by the automatic plan
    # (several split units meet at their barriers in the same launches); the
    # result is the unsplit run's and the oracle's
    require_gpu()
    descs = [sg.VbDesc(n=20011, T=0.8, seed=9, instance_id=k, graph_id=k, c=4.0) for k in range(3)]
    chunks = [4, 7]
    res = run_lib(descs, chunks, 16, threads_per_unit=64, split_members=0)
    ref = run_lib(descs, chunks, 16, threads_per_unit=64, split_members=1)
    assert_same(res, ref, "auto split vs unsplit")
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_vb(d, sum(chunks), 16), label="auto equal i=%d" % i)
