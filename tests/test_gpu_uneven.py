"""GPU parity of uneven VB batches (instances of very different sizes in one
context): several launch groups on their own streams, autotuned workgroup
sizes and hipGraph-replayed sweep chunks must all give the oracle's
trajectories exactly, including when eager work and measurements are
interleaved with graph replays."""
import numpy as np
import pytest

import paper_1906_11195_amd as sg
from paper_1906_11195_amd import workloads
from tests.gpu_util import assert_instance_equal, oracle_vb, require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS


def _small_uneven():
    # sizes log-uniform in [2^10, 2^16]: several launch groups
    return workloads.vb_uneven(count=12, lo=10, hi=16)


@pytest.mark.parametrize("autotune,graph", [(False, False), (True, True), (False, True)])
def test_uneven_batch_matches_oracle(autotune, graph):
    require_gpu()
    descs = _small_uneven()
    ctx = sg.sg_create_vb(descs, t_max=128, autotune=autotune, graph=graph)
    try:
        for k in (5, 32, 33):
            sg.sg_sweep(ctx, k)
        res = sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)
    for i, d in enumerate(descs):
        assert_instance_equal(res, i, oracle_vb(d, 70, 128), label="inst %d n=%d" % (i, d.n))


def test_graph_replays_interleaved_with_eager_work():
    import torch
    require_gpu()
    descs = _small_uneven()[:6]
    ctx = sg.sg_create_vb(descs, t_max=64, graph=True)
    x = torch.randn(1 << 20, device="cuda")
    try:
        for rep in range(4):
            sg.sg_sweep(ctx, 16)                   # same captured chunk replayed
            x = torch.sin(x) * 1.0001              # unrelated eager work on the stream
            torch.cuda.synchronize()
            res = sg.sg_measure(ctx, FLAGS)
            for i, d in enumerate(descs):
                assert_instance_equal(res, i, oracle_vb(d, 16 * (rep + 1), 64),
                                      label="replay %d inst %d" % (rep, i))
    finally:
        sg.sg_free(ctx)


def test_uneven_full_size_prefix_sampled():
    # The uneven configuration at full size: 1024 instances, N log-uniform in
    # [2^10, 2^20], 2 replicas, autotuned, graph-replayed; an 8-sweep prefix,
    # sampled instances (smallest, largest, and a few others) against the oracle.
    require_gpu()
    descs = workloads.vb_uneven()
    ctx = sg.sg_create_vb(descs, t_max=workloads.VB_UNEVEN_SWEEPS, autotune=True, graph=True)
    try:
        sg.sg_sweep(ctx, 4)
        sg.sg_sweep(ctx, 4)
        res = sg.sg_measure(ctx, sg.MEASURE_OBS)
    finally:
        sg.sg_free(ctx)
    ns = np.array([d.n for d in descs])
    G = res["gram"]
    for i in range(len(descs)):
        assert np.all(G[i, :, np.arange(5), np.arange(5)] == ns[i])
    for i in sorted({int(np.argmin(ns)), int(np.argmax(ns)), 0, 511, 1023}):
        ref = oracle_vb(descs[i], 8, workloads.VB_UNEVEN_SWEEPS)
        assert_instance_equal(res, i, ref, spins=False, label="inst %d n=%d" % (i, descs[i].n))
