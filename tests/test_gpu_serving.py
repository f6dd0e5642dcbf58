"""GPU test of the continuous-batching request loop: requests of both models
and different sizes, temperatures and lengths arrive close together, are
admitted as slots and memory free up, run concurrently on several streams,
and each result equals the same run alone (and, for a sample, the oracle),
also when the VB batches split their graphs over several workgroups."""
import numpy as np
import pytest

import paper_1906_11195_amd as sg
from paper_1906_11195_amd import serving, workloads
from tests.gpu_util import assert_instance_equal, oracle_sk, oracle_vb, require_gpu

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(11)
    reqs, t = [], 0.0
    for rid in range(14):
        t += rng.exponential(0.002)
        kind = "vb" if rid % 3 else "sk"
        n = int(2 ** rng.uniform(10, 13)) if kind == "vb" else int(2 ** rng.uniform(8, 10))
        T = float(rng.uniform(0.5, 0.9))
        sweeps = int(2 ** rng.integers(5, 9))
        reqs.append(workloads.Request(rid, t, kind, n, T, sweeps))
    return reqs


def test_served_results_equal_runs_alone():
    require_gpu()
    reqs = _requests()
    # small budget and few slots so that admission has to wait for memory
    server = serving.AgingServer(hbm_budget=24 << 20, max_active=5, chunk_sweeps=16, n_streams=3)
    results = server.run(reqs)
    assert sorted(r.rid for r in results) == [r.rid for r in reqs]
    by_id = {r.rid: r for r in results}
    for req in reqs:
        alone = serving.run_alone(req)
        got = by_id[req.rid].obs
        for key in ("bond", "overlap", "gram", "accepted"):
            assert np.array_equal(got[key], alone[key]), (req, key)
        assert np.array_equal(got["spins"][0], alone["spins"][0]), req
    stats = serving.latency_stats(results)
    assert stats["count"] == len(reqs) and stats["p99_ms"] >= stats["p50_ms"] > 0


def test_served_sample_matches_oracle():
    require_gpu()
    reqs = _requests()[:5]
    server = serving.AgingServer(hbm_budget=1 << 30, max_active=8, chunk_sweeps=32, n_streams=2)
    results = {r.rid: r for r in server.run(reqs)}
    for req in reqs[:3]:
        d = serving.descriptor(req)
        ref = (oracle_vb if req.kind == "vb" else oracle_sk)(d, req.sweeps, req.sweeps)
        assert_instance_equal(results[req.rid].obs, 0, ref, label="request %d" % req.rid)


def test_served_split_batches_equal_runs_alone():
    # VB runs large enough to be split over several workgroups, all arriving
    # together: with split_min_s = 0 every VB batch may split, and such
    # batches are created one at a time in admission order (longest first);
    # the results are those of the runs alone
    require_gpu()
    reqs = [workloads.Request(0, 0.0, "vb", 24000, 0.7, 128), workloads.Request(1, 0.0, "vb", 30000, 0.6, 64),
            workloads.Request(2, 0.0, "sk", 700, 0.5, 64), workloads.Request(3, 0.0, "vb", 20000, 0.8, 128),
            workloads.Request(4, 0.0, "vb", 28000, 0.9, 32)]
    server = serving.AgingServer(hbm_budget=1 << 30, max_active=8, chunk_sweeps=32, n_streams=3, split_min_s=0.0)
    results = {r.rid: r for r in server.run(reqs)}
    assert sorted(results) == [0, 1, 2, 3, 4]
    assert server._created == server._tickets == 3      # classes (vb, 128), (vb, 64), (vb, 32)
    for req in reqs:
        alone = serving.run_alone(req)
        got = results[req.rid].obs
        for key in ("bond", "overlap", "gram", "accepted"):
            assert np.array_equal(got[key], alone[key]), (req, key)
        assert np.array_equal(got["spins"][0], alone["spins"][0]), req
