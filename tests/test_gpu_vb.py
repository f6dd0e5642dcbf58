"""GPU parity of the VB path against the oracle (exact, all integers).

Covers the plain configuration in full, ragged sizes and tiny graphs,
explicit edge lists, T = inf and T = 0, aligned and given starts, graphs
shared by several temperatures, every chains-per-unit packing and several
workgroup sizes (results must not depend on them), sweeps split over calls,
and the full-size batched configuration on a prefix of sweeps with sampled
chains."""
import math

import numpy as np
import pytest

import oracle
import paper_1906_11195_amd as sg
from paper_1906_11195_amd import workloads
from tests.gpu_util import assert_instance_equal, oracle_vb, require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS


def run_lib(descs, n_sweeps, t_max, **kw):
    ctx = sg.sg_create_vb(descs, t_max=t_max, **kw)
    try:
        sg.sg_sweep(ctx, n_sweeps)
        return sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)


def test_vb_plain_full_run_matches_oracle():
    require_gpu()
    descs = workloads.vb_plain()
    res = run_lib(descs, workloads.VB_PLAIN_SWEEPS, workloads.VB_PLAIN_SWEEPS)
    ref = oracle_vb(descs[0], workloads.VB_PLAIN_SWEEPS, workloads.VB_PLAIN_SWEEPS)
    assert_instance_equal(res, 0, ref, label="vb plain")
    assert res["gram"][0, 0, 0, 0] == 1024


@pytest.mark.parametrize("n", [2, 3, 33, 100, 777, 1000, 4097])
def test_vb_ragged_sizes(n):
    require_gpu()
    d = sg.VbDesc(n=n, T=0.8, seed=11, instance_id=n, graph_id=1, c=4.0 if n > 3 else 1.0)
    res = run_lib([d], 70, 64)
    assert_instance_equal(res, 0, oracle_vb(d, 70, 64), label="n=%d" % n)


def test_vb_explicit_ring_and_limits_of_temperature():
    require_gpu()
    n = 501
    rng = np.random.default_rng(0)
    edges = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)
    J = rng.choice([-1, 1], size=n).astype(np.int8)
    descs = [sg.VbDesc(n=n, T=T, seed=5, instance_id=k, edges=edges, J=J)
             for k, T in enumerate([1.0, math.inf, 0.0])]
    res = run_lib(descs, 40, 32)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_vb(d, 40, 32), label="T=%s" % d.T)


def test_vb_aligned_and_given_starts():
    require_gpu()
    n = 3000
    rng = np.random.default_rng(1)
    s0 = rng.choice([-1, 1], size=(2, n)).astype(np.int8)
    descs = [sg.VbDesc(n=n, T=0.7, seed=8, instance_id=0, graph_id=2, start=sg.START_ALIGNED),
             sg.VbDesc(n=n, T=0.7, seed=8, instance_id=1, graph_id=2, start=sg.START_GIVEN, s0=s0)]
    res = run_lib(descs, 33, 32)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_vb(d, 33, 32), label="start=%d" % d.start)


@pytest.mark.parametrize("cpu,threads", [(0, 0), (1, 64), (2, 128), (4, 256), (8, 1024), (3, 192)])
def test_vb_shared_graph_any_packing(cpu, threads):
    # 2 graphs x 3 temperatures x 2 replicas; every packing of chains into
    # workgroups and every workgroup size gives the same trajectories.
    require_gpu()
    descs = workloads.vb_batched(n_graphs=2, n=2000)
    res = run_lib(descs, 65, 64, chains_per_unit=cpu, threads_per_unit=threads)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_vb(d, 65, 64), label="inst %d" % i)


def test_vb_sweeps_split_over_calls_and_batches():
    require_gpu()
    descs = workloads.vb_batched(n_graphs=3, n=1500)
    ctx = sg.sg_create_vb(descs, t_max=128)
    try:
        for k in (1, 2, 5, 0, 29, 91):
            sg.sg_sweep(ctx, k)
        a = sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)
    b = run_lib(descs[4:5], 128, 128)          # alone in its own context
    ref = oracle_vb(descs[4], 128, 128)
    assert_instance_equal(a, 4, ref, label="split")
    assert_instance_equal(b, 0, ref, label="alone")


def test_vb_measure_mid_run_has_zeros_beyond_reached_grid():
    require_gpu()
    d = workloads.vb_plain()[0]
    ctx = sg.sg_create_vb([d], t_max=4096)
    try:
        sg.sg_sweep(ctx, 100)
        r1 = sg.sg_measure(ctx, FLAGS)
        sg.sg_sweep(ctx, 28)
        r2 = sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)
    ref = oracle_vb(d, 100, 4096)
    assert_instance_equal(r1, 0, ref, label="t=100")
    assert r1["k_done"] == 8 and np.all(r1["bond"][0][:, 8:] == 0)
    assert_instance_equal(r2, 0, oracle_vb(d, 128, 4096), label="t=128")


def test_vb_batched_full_size_prefix_sampled():
    # The batched configuration at full size (256 graphs x 3 T x 2 replicas,
    # N = 65536, grid up to 2^20) in the launch shape the benchmark times, on
    # a 64-sweep prefix; sampled instances against the oracle, properties on all.
    require_gpu()
    descs = workloads.vb_batched()
    n_sw = 64
    ctx = sg.sg_create_vb(descs, t_max=workloads.VB_BATCHED_SWEEPS)
    try:
        sg.sg_sweep(ctx, n_sw)
        res = sg.sg_measure(ctx, sg.MEASURE_OBS)
    finally:
        sg.sg_free(ctx)
    K = 22
    assert res["k_done"] == 8
    G = res["gram"]
    assert np.all(G[:, :, np.arange(8), np.arange(8)] == 65536)
    assert np.array_equal(G, np.transpose(G, (0, 1, 3, 2)))
    assert np.all(G[:, :, 8:, :] == 0)
    # graphs 0, 127, 255 (maximum degree 15) and graphs 2 and 10 (a vertex of
    # degree 16 and 19: their chunks take the 8-bit count path)
    for i in (0, 6, 31, 383, 767):
        ref = oracle_vb(descs[i], n_sw, workloads.VB_BATCHED_SWEEPS)
        assert_instance_equal(res, i, ref, spins=False, label="inst %d" % i)
    assert res["bond"].shape == (768, 2, K)
