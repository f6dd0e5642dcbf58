"""GPU parity of the SK path against the oracle (exact, all integers).

Covers several samples with two clones through field recomputations, ragged
sizes (not multiples of the 64-spin block or of 16), T = inf and T = 0,
aligned and given starts, given couplings, sweeps split over calls, and the
full-size SK configuration on a prefix of sweeps with sampled chains, and
the largest supported sizes, and the sizes around the updaters' one-pass
capacity."""
import math

import numpy as np
import pytest

import oracle
import paper_1906_11195_amd as sg
from paper_1906_11195_amd import workloads
from tests.gpu_util import assert_instance_equal, oracle_sk, require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS


def run_lib(descs, n_sweeps, t_max, **kw):
    ctx = sg.sg_create_sk(descs, t_max=t_max, **kw)
    try:
        sg.sg_sweep(ctx, n_sweeps)
        return sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)


def test_sk_samples_through_recomputes():
    require_gpu()
    descs = workloads.sk_batch(n_samples=4, n=256)
    res = run_lib(descs, 200, 256)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_sk(d, 200, 256), label="sample %d" % i)


@pytest.mark.parametrize("n", [2, 5, 63, 65, 100, 130, 1000])
def test_sk_ragged_sizes(n):
    require_gpu()
    d = sg.SkDesc(n=n, T=0.5, seed=7, instance_id=n, graph_id=n, recompute_period=16)
    res = run_lib([d], 50, 32)
    assert_instance_equal(res, 0, oracle_sk(d, 50, 32), label="n=%d" % n)


def test_sk_temperature_limits_and_starts():
    require_gpu()
    n = 300
    rng = np.random.default_rng(3)
    s0 = rng.choice([-1, 1], size=(2, n)).astype(np.int8)
    J = oracle.sk_couplings(n, 9, 9)
    descs = [sg.SkDesc(n=n, T=math.inf, seed=1, instance_id=0, graph_id=1),
             sg.SkDesc(n=n, T=0.0, seed=1, instance_id=1, graph_id=1),
             sg.SkDesc(n=n, T=0.4, seed=1, instance_id=2, graph_id=1, start=sg.START_ALIGNED),
             sg.SkDesc(n=n, T=0.6, seed=1, instance_id=3, graph_id=2, start=sg.START_GIVEN, s0=s0, J=J)]
    res = run_lib(descs, 40, 32)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_sk(d, 40, 32), label="case %d" % i)


def test_sk_split_calls():
    require_gpu()
    descs = workloads.sk_batch(n_samples=2, n=512)
    ctx = sg.sg_create_sk(descs, t_max=128)
    try:
        for k in (3, 61, 1, 63):
            sg.sg_sweep(ctx, k)
        res = sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_sk(d, 128, 128), label="sample %d" % i)


def test_sk_full_size_prefix_sampled():
    # 64 samples x 2 replicas, N = 4096, T = 0.5, grid up to 2^16; 65 sweeps
    # (one exact recompute on the way); sampled chains against the oracle.
    require_gpu()
    descs = workloads.sk_batch()
    ctx = sg.sg_create_sk(descs, t_max=workloads.SK_SWEEPS)
    try:
        sg.sg_sweep(ctx, 65)
        res = sg.sg_measure(ctx, sg.MEASURE_OBS)
    finally:
        sg.sg_free(ctx)
    assert res["k_done"] == 8
    G = res["gram"]
    assert np.all(G[:, :, np.arange(8), np.arange(8)] == 4096)
    for i in (0, 37, 63):
        assert_instance_equal(res, i, oracle_sk(descs[i], 65, workloads.SK_SWEEPS), spins=False,
                              label="sample %d" % i)


@pytest.mark.parametrize("n", [16384, 32768])
def test_sk_largest_sizes(n):
    # The largest binary sizes: the fields fill most of the workgroup's LDS
    # (128 KiB at N = 32768), each coupling row spans 2-4 KiB, and the first
    # sweeps from a random start flip many spins per block.
    require_gpu()
    d = sg.SkDesc(n=n, T=0.5, seed=5, instance_id=0, graph_id=5, recompute_period=4)
    res = run_lib([d], 6, 8)
    assert_instance_equal(res, 0, oracle_sk(d, 6, 8), label="n=%d" % n)


@pytest.mark.parametrize("n", [4097, 7168, 7169, 8192])
def test_sk_updater_pass_boundaries(n):
    # The updater wavefronts apply a block's flips to 7168 fields per pass
    # (14 wavefronts x 64 lanes x 8 fields): one pass up to N = 7168, a
    # second, partly filled one above it; the serving workload's SK sizes
    # reach 8192.
    require_gpu()
    d = sg.SkDesc(n=n, T=0.5, seed=6, instance_id=1, graph_id=6, recompute_period=4)
    res = run_lib([d], 10, 16)
    assert_instance_equal(res, 0, oracle_sk(d, 10, 16), label="n=%d" % n)
