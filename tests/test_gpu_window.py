"""GPU parity of the windowed correlation (SG_OPT_WINDOW): the per-chain sums
of C(tau, t_w) over the minor-third intervals of tau = t_w + t, and their
term counts, equal the oracle's exactly (integers), for every chain packing,
LDS-resident and streamed adjacency, units split over several workgroups,
graph-replayed sweeps, runs over several calls and runs past t_max.  The
point observables are checked alongside."""
import concurrent.futures as cf
import math

import numpy as np
import pytest

import oracle
import paper_1906_11195_amd as sg
from tests.gpu_util import assert_instance_equal, require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS


def oracle_window(d, n_sweeps, t_max, tw_max):
    eu, ev, J = oracle.vb_instance(d.n, d.c, d.seed, d.graph_id)
    return oracle.vb_run(d.n, eu, ev, J, d.T, d.seed, d.instance_id, d.n_replicas, n_sweeps, t_max,
                         window_tw_max=tw_max)


def check(descs, chunks, t_max, tw_max, **kw):
    ctx = sg.sg_create_vb(descs, t_max=t_max, window_tw_max=tw_max, **kw)
    try:
        for k in chunks:
            sg.sg_sweep(ctx, k)
        res = sg.sg_measure(ctx, FLAGS)
        noalloc = sg.sg_measure_noalloc(ctx)
    finally:
        sg.sg_free(ctx)
    total = sum(chunks)
    with cf.ThreadPoolExecutor(max_workers=min(16, len(descs))) as ex:
        refs = list(ex.map(lambda d: oracle_window(d, total, t_max, tw_max), descs))
    assert np.array_equal(res["window_count"], refs[0]["window_count"]), "window counts"
    assert np.array_equal(noalloc["window_count"], refs[0]["window_count"]), "window counts (noalloc)"
    for i, ref in enumerate(refs):
        assert_instance_equal(res, i, ref, label="inst %d" % i)
        assert np.array_equal(res["window"][i], ref["window"]), "window sums, inst %d" % i
        assert np.array_equal(noalloc["window"][i], ref["window"]), "window sums (noalloc), inst %d" % i
    return res, refs


@pytest.mark.parametrize("n", [3001, 40007])
@pytest.mark.parametrize("cpu", [1, 2, 4, 8])
def test_window_every_packing(n, cpu):
    require_gpu()
    temps = [0.6, 1.2, math.inf, 0.9]
    descs = [sg.VbDesc(n=n, T=T, seed=31, instance_id=k, graph_id=2) for k, T in enumerate(temps)]
    res, refs = check(descs, [37, 90], 100, 16, chains_per_unit=cpu)
    # C(t_w, t_w) is not a term (tau > t_w); at T = inf, s(tau) = (-1)^(tau - t_w) s(t_w) exactly
    w = res["window"][2]
    cnt = res["window_count"]
    assert np.abs(w).sum() > 0 and cnt.sum() > 0


def test_window_split_units_graph_replay_and_past_t_max():
    require_gpu()
    descs = [sg.VbDesc(n=90001, T=T, seed=5, instance_id=k, graph_id=0) for k, T in enumerate([0.7, 1.0, 1.4])]
    # forced 3-member split; sweeps past t_max = 200 add nothing
    check(descs, [50, 101, 120], 200, 64, split_members=3, graph=True)


def test_window_waiting_times_off_the_grid_and_one_sweep_calls():
    require_gpu()
    descs = [sg.VbDesc(n=777, T=0.8, seed=8, instance_id=k, graph_id=k % 2, n_replicas=3) for k in range(4)]
    # tw_max = 5: waiting times 0, 1, 2, 4; t_max not a power of two
    check(descs, [1] * 9 + [40, 1, 250], 300, 5)
    # only t_w = 0
    check(descs[:1], [33], 33, 0)


def test_window_uneven_batch_with_autotune():
    require_gpu()
    rng = np.random.default_rng(12)
    ns = [int(2 ** (10 + 7 * u)) for u in rng.random(12)]
    descs = [sg.VbDesc(n=n, T=[0.6, 0.8, 1.0][k % 3], seed=4, instance_id=k, graph_id=k) for k, n in enumerate(ns)]
    check(descs, [64, 64], 128, 32, autotune=True, graph=True)


def test_window_full_batched_context_sampled():
    # the benchmark's windowed leg: all 768 instances (1536 chains, N = 65536,
    # 14 waiting times <= 2^12) in one context, a prefix of 40 sweeps,
    # sampled instances against the oracle
    require_gpu()
    from paper_1906_11195_amd import workloads
    descs = workloads.vb_batched()
    t_max, tw_max = workloads.VB_BATCHED_SWEEPS, 4096
    ctx = sg.sg_create_vb(descs, t_max=t_max, window_tw_max=tw_max)
    try:
        sg.sg_sweep(ctx, 17)
        sg.sg_sweep(ctx, 23)
        res = sg.sg_measure(ctx, sg.MEASURE_OBS)
    finally:
        sg.sg_free(ctx)
    picks = [0, 383, 767]
    with cf.ThreadPoolExecutor(max_workers=3) as ex:
        refs = list(ex.map(lambda i: oracle_window(descs[i], 40, t_max, tw_max), picks))
    assert np.array_equal(res["window_count"], refs[0]["window_count"])
    for i, ref in zip(picks, refs):
        assert np.array_equal(res["window"][i], ref["window"]), "window sums, inst %d" % i
        assert np.array_equal(res["gram"][i], ref["gram"]) and np.array_equal(res["bond"][i], ref["bond"])
