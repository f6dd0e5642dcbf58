"""Pins of the oracle's windowed correlation (the paper's estimator: C(t_w + t,
t_w) averaged over geometric intervals of ratio 2^(1/4) in the time t_w + t;
Results and discussion, and the SI section on the extrapolation to large
sizes and times).

  * interval index of tau: Python's exact big-integer floor(log2 tau^4)
    against the closed forms at powers of two, and the interval edges
    against 2^(m/4) in floating point away from ties;
  * brute force: every sweep's configuration obtained by re-running the
    oracle to that time, overlaps with numpy, summed per interval;
  * T = inf: s(tau) = (-1)^tau s(0), so every overlap is +-N by parity;
  * counts: each waiting time sees every tau in (t_w, t_done] exactly once.
"""
import math

import numpy as np
import pytest

import oracle


def py_bin(tau):
    return (tau ** 4).bit_length() - 1


def test_interval_index():
    for j in range(0, 31):
        assert oracle.window_bin(1 << j) == 4 * j
        if j >= 3:     # (1 - 2^-j)^4 >= 1/2 from j = 3 on
            assert oracle.window_bin((1 << j) - 1) == 4 * j - 1
    for tau in list(range(1, 5000)) + [2 ** 31 - 1, 2 ** 32 - 1, 3 ** 19, 10 ** 9 + 7]:
        assert oracle.window_bin(tau) == py_bin(tau), tau
    # edges: tau is in interval m iff 2^(m/4) <= tau < 2^((m+1)/4)
    for tau in range(1, 20000):
        m = oracle.window_bin(tau)
        lo, hi = 2.0 ** (m / 4.0), 2.0 ** ((m + 1) / 4.0)
        assert lo * (1 - 1e-12) <= tau < hi * (1 + 1e-12)


def test_waiting_times_are_the_grid_prefix():
    assert oracle.window_tw_count(1 << 20, 4096) == 14      # 0, 1, 2, ..., 4096
    assert oracle.window_tw_count(100, 0) == 1
    assert oracle.window_tw_count(100, 3) == 3               # 0, 1, 2
    assert oracle.window_tw_count(8, 1000) == 5              # the whole grid


def test_window_brute_force_from_reruns():
    n, T, t_max, tw_max = 150, 0.8, 40, 8
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=6, graph_id=2)
    full = oracle.vb_run(n, eu, ev, J, T, 6, 3, 2, t_max, t_max, window_tw_max=tw_max)
    conf = [oracle.vb_run(n, eu, ev, J, T, 6, 3, 2, tau, t_max)["spins"].astype(np.int64)
            for tau in range(t_max + 1)]
    tws = [t for t in full["times"] if t <= tw_max]
    M = py_bin(t_max) + 1
    want = np.zeros((2, len(tws), M), np.int64)
    cnt = np.zeros((len(tws), M), np.int64)
    for k, tw in enumerate(tws):
        for tau in range(tw + 1, t_max + 1):
            m = py_bin(tau)
            want[:, k, m] += np.sum(conf[tau] * conf[tw], axis=1)
            cnt[k, m] += 1
    assert np.array_equal(full["window"], want)
    assert np.array_equal(full["window_count"], cnt)
    # C(tau, t_w) <= 1 on average and the interval holding tau = t_w + 1 is
    # dominated by large correlations
    C = full["window"] / np.maximum(cnt, 1) / n
    assert np.all(np.abs(C) <= 1)


def test_window_infinite_temperature_closed_form():
    n, t_max, tw_max = 64, 100, 16
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=2, graph_id=0)
    o = oracle.vb_run(n, eu, ev, J, math.inf, 2, 0, 1, 70, t_max, window_tw_max=tw_max)
    tws = [t for t in o["times"] if t <= tw_max]
    for k, tw in enumerate(tws):
        for m in range(o["window"].shape[2]):
            taus = [tau for tau in range(tw + 1, 71) if py_bin(tau) == m]
            assert o["window_count"][k, m] == len(taus)
            assert o["window"][0, k, m] == sum(n if (tau - tw) % 2 == 0 else -n for tau in taus)


@pytest.mark.parametrize("n_sweeps", [0, 1, 33, 500])
def test_window_counts_cover_every_time_once(n_sweeps):
    n, t_max, tw_max = 40, 300, 64
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=1, graph_id=1)
    o = oracle.vb_run(n, eu, ev, J, 0.7, 1, 0, 1, n_sweeps, t_max, window_tw_max=tw_max)
    done = min(n_sweeps, t_max)
    tws = [t for t in o["times"] if t <= tw_max]
    for k, tw in enumerate(tws):
        assert o["window_count"][k].sum() == max(0, done - tw)
