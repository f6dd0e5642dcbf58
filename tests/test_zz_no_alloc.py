"""GPU tests of sg_measure_noalloc, the measurement entry point that
allocates no memory (its kernels stage results in a fixed device array):
its observables equal sg_measure's exactly, on two calls in a row with the
second context smaller than the first (the shared array then still holds the
first call's values), for VB and SK contexts; oversized contexts and
requests for spins are refused."""
import ctypes

import numpy as np
import pytest

import paper_1906_11195_amd as sg
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

KEYS = ("times", "bond", "overlap", "gram", "accepted")


def _same(a, b, label):
    assert a["k_done"] == b["k_done"] and a["t_done"] == b["t_done"], label
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), "%s: %s differs" % (label, k)


def _vb_pair(descs, sweeps, t_max):
    ctx = sg.sg_create_vb(descs, t_max=t_max)
    try:
        sg.sg_sweep(ctx, sweeps)
        ref = sg.sg_measure(ctx, sg.MEASURE_OBS)
        got = sg.sg_measure_noalloc(ctx)
        again = sg.sg_measure(ctx, sg.MEASURE_OBS)
    finally:
        sg.sg_free(ctx)
    return ref, got, again


def test_noalloc_vb_equals_measure_on_two_calls():
    require_gpu()
    big = [sg.VbDesc(n=3001, T=T, seed=11, instance_id=k, graph_id=k // 2)
           for k, T in enumerate([0.6, 0.8, 1.2, 0.8, float("inf")])]
    ref, got, again = _vb_pair(big, 100, 256)
    _same(got, ref, "VB first call")
    _same(again, ref, "VB after the variant")
    assert ref["k_done"] == 8 and np.abs(ref["gram"]).sum() > 0
    # smaller: fewer chains and grid times; stale entries must not show
    small = [sg.VbDesc(n=500, T=0.7, seed=12, instance_id=k, graph_id=0, n_replicas=3) for k in range(2)]
    ref, got, _ = _vb_pair(small, 10, 16)
    _same(got, ref, "VB second, smaller call")
    assert ref["k_done"] == 5 and got["gram"].shape == (2, 3, 6, 6)
    assert np.all(got["gram"][:, :, 5, :] == 0) and np.all(got["bond"][:, :, 5] == 0)


def test_noalloc_sk_equals_measure_on_two_calls():
    require_gpu()
    for descs, sweeps, t_max in (
            ([sg.SkDesc(n=300, T=0.5, seed=3, instance_id=k, graph_id=k) for k in range(3)], 70, 128),
            ([sg.SkDesc(n=130, T=0.9, seed=4, instance_id=0, graph_id=0)], 5, 4)):
        ctx = sg.sg_create_sk(descs, t_max=t_max)
        try:
            sg.sg_sweep(ctx, sweeps)
            ref = sg.sg_measure(ctx, sg.MEASURE_OBS)
            got = sg.sg_measure_noalloc(ctx)
        finally:
            sg.sg_free(ctx)
        _same(got, ref, "SK n=%d" % descs[0].n)


def test_noalloc_refuses_oversized_contexts_and_spins():
    require_gpu()
    # 1120 chains with 32 grid times need 1120 * 32 * 33 + 140 * 28 * 32
    # staging entries, more than the 2^20 of the fixed array
    descs = [sg.VbDesc(n=16, T=1.0, seed=1, instance_id=k, graph_id=k, n_replicas=8) for k in range(140)]
    ctx = sg.sg_create_vb(descs, t_max=1 << 30)
    try:
        sg.sg_sweep(ctx, 3)
        assert sg.sg_measure_noalloc(ctx, check=False)["status"] == sg.SG_ENOTSUP
        o = sg._Obs()
        spins = np.zeros(16 * 8 * 140, np.int8)
        o.spins = ctypes.c_void_p(spins.ctypes.data)
        assert sg.library().sg_measure_noalloc(ctx.ptr, ctypes.byref(o), None) == sg.SG_EINVAL
        assert sg.sg_measure(ctx, sg.MEASURE_OBS)["k_done"] == 3
    finally:
        sg.sg_free(ctx)
