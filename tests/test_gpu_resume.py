"""Checkpoint and resume (sg_opts.t_start): a run of t1 sweeps whose spins
are exported with sg_measure(SG_MEASURE_SPINS) and passed as the start
configurations of a new context with t_start = t1, swept t2 more, equals the
uninterrupted run of t1 + t2 sweeps bit for bit: final spins, accepted flips
(first part + resumed part), and every observable of the grid times after
t1 (bond sums, overlaps, Gram entries, also against the start snapshot when
t1 is itself a grid time).  The random streams are counter-based and keyed
by the sweep index (Methods), so nothing but the spins and the time has to be
carried over.  The uninterrupted run is itself compared with the oracle.
Per-chain VB (t1 a grid time or not; graph replay, autotuned launch groups,
units split over two workgroups), multispin VB, binary SK (t1 off the
recompute period) and real-coupling SK (t1 on it; off it is refused)."""
import dataclasses

import numpy as np
import pytest

import oracle
import paper_1906_11195_amd as sg
from paper_1906_11195_amd import workloads
from paper_1906_11195_amd.workloads import gaussian_couplings, random_regular_edges
from tests.gpu_util import assert_instance_equal, oracle_sk, oracle_vb, require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS


def run(kind, descs, chunks, t_max, **kw):
    create = sg.sg_create_vb if kind == "vb" else sg.sg_create_sk
    ctx = create(descs, t_max=t_max, **kw)
    try:
        for k in chunks:
            sg.sg_sweep(ctx, k)
        return sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)


def split_equals_whole(kind, descs, t1, t2, t_max, **kw):
    whole = run(kind, descs, [t1, t2], t_max, **kw)
    first = run(kind, descs, [t1], t_max, **kw)
    again = [dataclasses.replace(d, start=sg.START_GIVEN, s0=first["spins"][i]) for i, d in enumerate(descs)]
    rest = run(kind, again, [t2], t_max, t_start=t1, **kw)

    times = list(whole["times"])
    K = len(times)
    want_times = [t1] + [t if t > t1 else -1 for t in times[1:]]
    assert list(rest["times"]) == want_times
    assert rest["t_done"] == whole["t_done"] == t1 + t2
    assert rest["k_done"] == whole["k_done"]
    kd = whole["k_done"]
    after = [k for k in range(1, kd) if times[k] > t1]          # slots both runs took
    k_t1 = times.index(t1) if t1 in times else None            # the whole run's slot of time t1
    skipped = [k for k in range(1, K) if want_times[k] < 0]
    for i in range(len(descs)):
        lab = "instance %d" % i
        assert np.array_equal(rest["spins"][i], whole["spins"][i]), lab + " spins"
        assert np.array_equal(first["accepted"][i] + rest["accepted"][i], whole["accepted"][i]), lab + " accepted"
        for key in ("bond", "overlap") + (("bond_real",) if "bond_real" in whole else ()):
            w, r = np.asarray(whole[key][i]), np.asarray(rest[key][i])
            if w.size == 0:
                continue
            assert np.array_equal(r[..., after], w[..., after]), lab + " " + key
            if k_t1 is not None:
                assert np.array_equal(r[..., 0], w[..., k_t1]), lab + " " + key + " at t1"
            assert np.all(r[..., skipped] == 0), lab + " " + key + " slots not taken"
        G, W = np.asarray(rest["gram"][i]), np.asarray(whole["gram"][i])
        assert np.array_equal(G[:, after][:, :, after], W[:, after][:, :, after]), lab + " gram"
        if k_t1 is not None:
            assert np.array_equal(G[:, 0, after], W[:, k_t1, after]), lab + " gram with t1"
            assert np.array_equal(G[:, 0, 0], W[:, k_t1, k_t1]), lab + " gram at t1"
        assert np.all(G[:, skipped, :] == 0) and np.all(G[:, :, skipped] == 0), lab + " gram slots not taken"
    return whole


@pytest.mark.parametrize("t1,t2", [(256, 300), (100, 200)])
def test_vb_resume(t1, t2):
    require_gpu()
    descs = [sg.VbDesc(n=1000, T=T, seed=11, instance_id=i, graph_id=3, n_replicas=2)
             for i, T in enumerate((0.6, 1.0, 1.5))]
    whole = split_equals_whole("vb", descs, t1, t2, 1024)
    for i, d in enumerate(descs):
        assert_instance_equal(whole, i, oracle_vb(d, t1 + t2, 1024), label="whole run, instance %d" % i)


def test_vb_multispin_resume():
    require_gpu()
    n = 1200
    e, _ = random_regular_edges(n, 4, seed=9, bipartite=True)
    rng = np.random.default_rng(4)
    descs = [sg.VbDesc(n=n, T=(0.7, 1.1)[k % 2], seed=4, instance_id=k, edges=e,
                       J=rng.choice([-1, 1], size=len(e)).astype(np.int8), n_replicas=1) for k in range(20)]
    whole = split_equals_whole("vb", descs, 64, 70, 256, multispin=True)
    for i in (0, 7, 19):
        assert_instance_equal(whole, i, oracle_vb(descs[i], 134, 256), label="whole run, instance %d" % i)


def test_sk_resume_off_the_recompute_period():
    require_gpu()
    descs = workloads.sk_batch(n_samples=2, n=300)
    descs = [dataclasses.replace(d, recompute_period=16) for d in descs]
    whole = split_equals_whole("sk", descs, 40, 90, 128)
    for i, d in enumerate(descs):
        assert_instance_equal(whole, i, oracle_sk(d, 130, 128), label="whole run, sample %d" % i)


def test_sk_real_couplings_resume():
    require_gpu()
    n = 200
    descs = [sg.SkDesc(n=n, T=0.5, seed=2, instance_id=i, graph_id=i, recompute_period=16,
                       Jf=gaussian_couplings(n, 30 + i)) for i in range(2)]
    whole = split_equals_whole("sk", descs, 32, 40, 128)
    for i, d in enumerate(descs):
        ref = oracle.skg_run(d.n, d.Jf, d.T, d.seed, d.instance_id, d.n_replicas, 72, 128, period=16)
        assert np.array_equal(whole["spins"][i], ref["spins"])
        assert np.array_equal(whole["gram"][i], ref["gram"])
    # off the recompute period the fields would not be the uninterrupted run's
    with pytest.raises(sg.SgError) as e:
        sg.sg_create_sk(descs, t_max=128, t_start=20)
    assert e.value.code == sg.SG_EINVAL


@pytest.mark.parametrize("opts", [dict(graph=True), dict(autotune=True), dict(split_members=2)],
                         ids=["graph", "autotune", "split"])
def test_vb_resume_launch_paths(opts):
    # the resumed context's device sweep counter starts at t_start on every
    # launch path: captured graph replays, autotuned launch groups (their
    # trial launches restore the state), units split over two workgroups
    require_gpu()
    descs = [sg.VbDesc(n=20000, T=T, seed=13, instance_id=i, graph_id=4, n_replicas=2)
             for i, T in enumerate((0.7, 1.3))]
    whole = split_equals_whole("vb", descs, 128, 150, 512, **opts)
    for i, d in enumerate(descs):
        assert_instance_equal(whole, i, oracle_vb(d, 278, 512), label="whole run, instance %d" % i)
