"""Pins for the oracle's Metropolis dynamics and observables (CPU only).

Each check is fixed by the mathematics rather than by the oracle itself:
exact master-equation transients and Boltzmann equilibrium on tiny graphs
(tests/brute.py, independent numpy code), the T = inf and T = 0 limits, gauge
and global-flip symmetry, equality of sequential and class-synchronous sweeps
(proper colouring), closed-form paramagnetic energies, and observables
recomputed from returned configurations.
"""
import math

import numpy as np
import pytest

import oracle
from tests import brute


def _ring_with_chords(n, seed):
    rng = np.random.default_rng(seed)
    eu = list(range(n))
    ev = [(i + 1) % n for i in range(n)]
    # a few chords so that the graph is frustrated and non-bipartite
    eu += [0, 1, 2]
    ev += [n // 2, n // 2 + 2, n - 2]
    J = rng.choice([-1, 1], size=len(eu)).astype(np.int8)
    return np.array(eu, np.int32), np.array(ev, np.int32), J


def _vb_many(n, eu, ev, J, T, n_inst, n_sweeps, t_max, seed=11):
    bonds = []
    for inst in range(n_inst):
        o = oracle.vb_run(n, eu, ev, J, T, seed, inst, 1, n_sweeps, t_max)
        bonds.append(o["bond"][0])
    return np.array(bonds, dtype=np.float64), o["times"]


@pytest.mark.parametrize("T", [0.7, 1.5])
def test_vb_transient_energy_matches_master_equation(T):
    # Exact E[B(t)] from the uniform random start, propagated with the
    # one-sweep transition operator built from the definition, against the
    # mean over many oracle instances.
    n = 8
    eu, ev, J = _ring_with_chords(n, seed=1)
    A = brute.coupling_matrix(n, eu, ev, J)
    S = brute.states(n)
    B = brute.bond_sum(S, A).astype(float)
    order = brute.sweep_order(brute.greedy_colour(n, A), A)
    n_inst, t_max = 6000, 8
    bonds, times = _vb_many(n, eu, ev, J, T, n_inst, t_max, t_max)
    dist = np.full(1 << n, 1.0 / (1 << n))
    t_now = 0
    for k, t in enumerate(times):
        while t_now < t:
            dist = brute.sweep(dist, S, A, order, T)
            t_now += 1
        mean_exact = float(dist @ B)
        var_exact = float(dist @ (B - mean_exact) ** 2)
        se = math.sqrt(max(var_exact, 1e-12) / n_inst)
        z = (bonds[:, k].mean() - mean_exact) / se
        assert abs(z) < 5.0, (t, bonds[:, k].mean(), mean_exact, z)


def test_order_inside_a_colour_class_does_not_change_the_law():
    # The reading that visits each colour class by decreasing degree (then
    # id): the spins of a class are pairwise unconnected, so their single-spin
    # updates commute and the one-sweep transition operator (the law of the
    # dynamics, Eq. 3 with the Metropolis rule) is the same for every order
    # inside the classes.  The operator for the oracle's order equals the
    # one for id order and for random in-class permutations, column by column
    # (each basis state propagated exactly); changing the order of the classes
    # does change it (control).
    n, T = 8, 0.9
    eu, ev, J = _ring_with_chords(n, seed=5)
    A = brute.coupling_matrix(n, eu, ev, J)
    S = brute.states(n)
    colour, ncol = oracle.greedy_colour(n, eu, ev)
    assert ncol >= 3
    assert np.all(colour[eu] != colour[ev])

    def operator(order):
        cols = []
        for s0 in range(1 << n):
            e = np.zeros(1 << n)
            e[s0] = 1.0
            cols.append(brute.sweep(e, S, A, list(order), T))
        return np.stack(cols, axis=1)

    base = operator(oracle.sweep_order(colour, ncol, oracle.degrees(n, eu, ev)))
    assert np.allclose(base.sum(axis=0), 1.0, atol=1e-12)
    assert np.allclose(operator(sorted(range(n), key=lambda v: (colour[v], v))), base, atol=1e-13)
    rng = np.random.default_rng(2)
    for _ in range(3):
        perm = sorted(range(n), key=lambda v: (colour[v], rng.random()))
        assert np.allclose(operator(perm), base, atol=1e-13)
    reversed_classes = sorted(range(n), key=lambda v: (-colour[v], v))
    assert not np.allclose(operator(reversed_classes), base, atol=1e-6)


def test_vb_equilibrium_is_boltzmann():
    # Long runs sample the Boltzmann distribution exp(-H/T) (Eq. 3 with the
    # Metropolis rule); compare state frequencies by chi^2 and check pi P = pi.
    from scipy import stats
    n, T = 6, 1.2
    eu, ev, J = _ring_with_chords(n, seed=3)
    A = brute.coupling_matrix(n, eu, ev, J)
    S = brute.states(n)
    order = brute.sweep_order(brute.greedy_colour(n, A), A)
    pi = brute.boltzmann(S, A, T)
    assert np.allclose(brute.sweep(pi, S, A, order, T), pi, atol=1e-12)
    counts = np.zeros(1 << n)
    for inst in range(3000):
        o = oracle.vb_run(n, eu, ev, J, T, 21, inst, 2, 32, 32)
        for s in o["spins"]:
            counts[int(np.sum(((1 - s.astype(np.int64)) // 2) << np.arange(n)))] += 1
    chi2, pval = stats.chisquare(counts, pi * counts.sum())
    assert pval > 1e-4


def test_vb_infinite_temperature_alternates():
    n = 1024
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=1, graph_id=0)
    o = oracle.vb_run(n, eu, ev, J, math.inf, 1, 0, 2, 64, 64)
    start = oracle.vb_run(n, eu, ev, J, math.inf, 1, 0, 2, 0, 64)
    s0 = start["spins"]
    assert np.array_equal(o["spins"], s0)                    # even number of sweeps
    assert np.all(o["accepted"] == 64 * n)
    assert np.all(o["bond"] == o["bond"][:, :1])             # B is invariant under s -> -s
    for k, t in enumerate(o["times"]):
        for l, u in enumerate(o["times"]):
            assert np.all(o["gram"][:, k, l] == (n if (t - u) % 2 == 0 else -n))
    assert np.all(o["overlap"] == o["overlap"][:, :1])


def test_vb_zero_temperature_energy_never_rises():
    n = 2048
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=1, graph_id=3)
    s = oracle.vb_run(n, eu, ev, J, 0.0, 5, 0, 1, 0, 0)["spins"]
    prev = None
    for _ in range(30):
        o = oracle.vb_run(n, eu, ev, J, 0.0, 5, 0, 1, 1, 1, start=oracle.START_GIVEN, s0=s)
        b0, b1 = o["bond"][0]
        assert b1 >= b0
        if prev is not None:
            assert b0 == prev
        prev = b1
        s = o["spins"]


def test_vb_gauge_and_global_flip_invariance():
    n, T = 4096, 0.8
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=1, graph_id=0)
    rng = np.random.default_rng(0)
    s0 = rng.choice([-1, 1], size=(2, n)).astype(np.int8)
    g = rng.choice([-1, 1], size=n).astype(np.int8)
    a = oracle.vb_run(n, eu, ev, J, T, 1, 0, 2, 100, 128, start=oracle.START_GIVEN, s0=s0)
    Jg = (J * g[eu] * g[ev]).astype(np.int8)
    b = oracle.vb_run(n, eu, ev, Jg, T, 1, 0, 2, 100, 128, start=oracle.START_GIVEN,
                      s0=(s0 * g).astype(np.int8))
    assert np.array_equal(b["spins"], a["spins"] * g)
    for key in ("bond", "overlap", "gram", "accepted"):
        assert np.array_equal(a[key], b[key]), key
    c = oracle.vb_run(n, eu, ev, J, T, 1, 0, 2, 100, 128, start=oracle.START_GIVEN,
                      s0=(-s0).astype(np.int8))
    assert np.array_equal(c["spins"], -a["spins"])
    assert np.array_equal(c["gram"], a["gram"]) and np.array_equal(c["bond"], a["bond"])


def test_vb_class_synchronous_equals_sequential():
    n, T = 4096, 0.8
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=7, graph_id=2)
    a = oracle.vb_run(n, eu, ev, J, T, 7, 5, 2, 64, 64, mode=0)
    b = oracle.vb_run(n, eu, ev, J, T, 7, 5, 2, 64, 64, mode=1)
    for key in ("spins", "bond", "overlap", "gram", "accepted"):
        assert np.array_equal(a[key], b[key]), key


def test_vb_observables_recomputed_from_configurations():
    n, T, t_max = 1024, 0.8, 256
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=1, graph_id=0)
    o = oracle.vb_run(n, eu, ev, J, T, 1, 0, 2, t_max, t_max)
    K = len(o["times"])
    assert o["k_done"] == K
    G = o["gram"]
    assert np.all(G[:, np.arange(K), np.arange(K)] == n)      # C(t, t) = 1
    assert np.array_equal(G, np.transpose(G, (0, 2, 1)))
    for r in range(2):
        assert np.linalg.eigvalsh(G[r].astype(float)).min() > -1e-6 * n
    # last grid time is the final configuration
    s = o["spins"].astype(np.int64)
    for r in range(2):
        assert o["bond"][r, -1] == int(np.sum(J * s[r, eu] * s[r, ev]))
    assert o["overlap"][0, -1] == int(np.sum(s[0] * s[1]))
    # C(0, t_max) from the random start rebuilt from the INIT stream
    colour, ncol = oracle.greedy_colour(n, eu, ev)
    order = oracle.sweep_order(colour, ncol, oracle.degrees(n, eu, ev))
    for r in range(2):
        init = np.zeros(n, np.int64)
        init[order] = [oracle.init_spin(1, 0, r, p) for p in range(n)]
        assert G[r, 0, -1] == int(np.sum(init * s[r]))
        assert G[r, -1, 0] == G[r, 0, -1]
    # 2 B = sum_i s_i h_i
    h = np.zeros(n, np.int64)
    np.add.at(h, eu, J * s[0, ev])
    np.add.at(h, ev, J * s[0, eu])
    assert 2 * o["bond"][0, -1] == int(np.sum(s[0] * h))


def test_vb_gram_equals_library_matmul_of_snapshots():
    # Gram from the oracle against numpy's integer S^T S of snapshots obtained
    # by re-running to each grid time.
    n, T, t_max = 512, 0.8, 16
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=3, graph_id=1)
    full = oracle.vb_run(n, eu, ev, J, T, 3, 9, 1, t_max, t_max)
    snaps = [oracle.vb_run(n, eu, ev, J, T, 3, 9, 1, int(t), t_max)["spins"][0]
             for t in full["times"]]
    S = np.stack(snaps).astype(np.int64)
    assert np.array_equal(S @ S.T, full["gram"][0])


def test_ring_equilibrium_energy_closed_form():
    # 1-D ring with +-J couplings: <J s_i s_{i+1}> = (t + t^{N-1}) / (1 + t^N),
    # t = tanh(beta); gauge-equivalent to the ferromagnetic ring.
    n, T = 1000, 1.0
    rng = np.random.default_rng(4)
    eu = np.arange(n, dtype=np.int32)
    ev = ((np.arange(n) + 1) % n).astype(np.int32)
    J = rng.choice([-1, 1], size=n).astype(np.int8)
    t = math.tanh(1.0 / T)
    e_exact = -(t + t ** (n - 1)) / (1 + t ** n)
    vals = []
    for inst in range(8):
        o = oracle.vb_run(n, eu, ev, J, T, 2, inst, 2, 1024, 1024)
        vals.extend((-o["bond"][:, -4:] / n).ravel())
    vals = np.array(vals)
    assert abs(vals.mean() - e_exact) < 5 * vals.std() / math.sqrt(len(vals)) + 2e-3


def test_er_paramagnet_energy_closed_form():
    # Above T_c on a locally tree-like graph each bond is independent:
    # e = -(M/N) tanh(beta) = -(c/2) tanh(beta).
    n, c, T = 8192, 4.0, 3.0
    eu, ev, J = oracle.vb_instance(n, c, seed=6, graph_id=0)
    o = oracle.vb_run(n, eu, ev, J, T, 6, 0, 2, 512, 512)
    e = -o["bond"][:, -3:].mean() / n
    assert abs(e - (-(c / 2) * math.tanh(1 / T))) < 0.01


def test_vb_quench_ages():
    # Qualitative relaxation after a quench (main text, Fig. 1 discussion):
    # C(tw+t, tw) decreases with t at fixed tw and the energy relaxes.
    n, T, t_max = 8192, 0.8, 1024
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=1, graph_id=0)
    o = oracle.vb_run(n, eu, ev, J, T, 1, 0, 2, t_max, t_max)
    C = o["gram"].mean(axis=0) / n
    times = list(o["times"])
    k4, k16 = times.index(4), times.index(16)
    assert np.all(np.diff(C[k4, k4:]) < 0)
    assert np.all(np.diff(C[k16, k16:]) < 0)
    assert np.all(np.diff(o["bond"].mean(axis=0)[1:]) > -0.02 * n)   # energy relaxes


# ---------------------------------------------------------------------------
# SK
# ---------------------------------------------------------------------------

def test_sk_incremental_fields_equal_direct():
    n, T = 384, 0.5
    J = oracle.sk_couplings(n, seed=3, graph_id=0)
    a = oracle.sk_run(n, J, T, 3, 0, 2, 40, 64, direct=True)
    b = oracle.sk_run(n, J, T, 3, 0, 2, 40, 64, direct=False)
    for key in ("spins", "bond", "overlap", "gram", "accepted"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("T", [0.6, 2.0])
def test_sk_transient_energy_matches_master_equation(T):
    n = 7
    J = oracle.sk_couplings(n, seed=5, graph_id=2)
    A = J.astype(np.int64)
    S = brute.states(n)
    B = brute.bond_sum(S, A).astype(float)
    scale = 1.0 / math.sqrt(n)
    n_inst, t_max = 6000, 8
    bonds = np.array([oracle.sk_run(n, J, T, 17, inst, 1, t_max, t_max)["bond"][0]
                      for inst in range(n_inst)], float)
    times = oracle.grid(t_max)
    dist = np.full(1 << n, 1.0 / (1 << n))
    t_now = 0
    for k, t in enumerate(times):
        while t_now < t:
            dist = brute.sweep(dist, S, A, list(range(n)), T, scale)
            t_now += 1
        m = float(dist @ B)
        se = math.sqrt(max(float(dist @ (B - m) ** 2), 1e-12) / n_inst)
        assert abs(bonds[:, k].mean() - m) < 5 * se, (t, bonds[:, k].mean(), m)


def test_sk_gauge_flip_and_infinite_temperature():
    n, T = 256, 0.5
    J = oracle.sk_couplings(n, seed=1, graph_id=1)
    rng = np.random.default_rng(2)
    s0 = rng.choice([-1, 1], size=(2, n)).astype(np.int8)
    g = rng.choice([-1, 1], size=n).astype(np.int8)
    a = oracle.sk_run(n, J, T, 1, 4, 2, 64, 64, start=oracle.START_GIVEN, s0=s0)
    Jg = (J * g[:, None] * g[None, :]).astype(np.int8)
    b = oracle.sk_run(n, Jg, T, 1, 4, 2, 64, 64, start=oracle.START_GIVEN, s0=(s0 * g).astype(np.int8))
    assert np.array_equal(b["spins"], a["spins"] * g)
    assert np.array_equal(a["gram"], b["gram"]) and np.array_equal(a["bond"], b["bond"])
    c = oracle.sk_run(n, J, math.inf, 1, 4, 2, 9, 16, start=oracle.START_GIVEN, s0=s0)
    assert np.array_equal(c["spins"], -s0)
    assert np.all(c["accepted"] == 9 * n)
    s = a["spins"].astype(np.int64)
    assert a["bond"][0, -1] == int(s[0] @ np.triu(J.astype(np.int64), 1) @ s[0])


def test_sk_paramagnet_energy_closed_form():
    # T > 1: e = -beta/2 in the large-N limit (here -beta (N-1) / (2N)).
    n, T = 512, 2.0
    J = oracle.sk_couplings(n, seed=8, graph_id=0)
    vals = []
    for inst in range(4):
        o = oracle.sk_run(n, J, T, 8, inst, 2, 128, 128)
        vals.extend((-o["bond"][:, -2:] / math.sqrt(n) / n).ravel())
    assert abs(np.mean(vals) - (-(1 / T) * (n - 1) / (2 * n))) < 0.02


def test_sk_aligned_start():
    n = 128
    J = oracle.sk_couplings(n, seed=1, graph_id=0)
    o = oracle.sk_run(n, J, 0.5, 1, 0, 2, 0, 0, start=oracle.START_ALIGNED)
    assert np.all(o["spins"] == 1)
    assert o["bond"][0, 0] == int(np.triu(J.astype(np.int64), 1).sum())


def test_sk_observables_recomputed_from_configurations():
    # Bond, overlap and Gram of the SK run against values recomputed with
    # numpy from the configurations themselves: snapshots obtained by
    # re-running the oracle to each grid time, the start rebuilt from the
    # INIT stream (SK visits i = 0..N-1, so position = vertex).
    n, T, t_max = 200, 0.5, 32
    J = oracle.sk_couplings(n, seed=4, graph_id=3)
    A = np.triu(J.astype(np.int64), 1)
    full = oracle.sk_run(n, J, T, 4, 6, 2, t_max, t_max)
    K = len(full["times"])
    assert full["k_done"] == K
    snaps = np.stack([oracle.sk_run(n, J, T, 4, 6, 2, int(t), t_max)["spins"] for t in full["times"]])
    S = snaps.astype(np.int64)                     # [K][replica][n]
    for r in range(2):
        G = S[:, r, :] @ S[:, r, :].T
        assert np.array_equal(G, full["gram"][r])
        assert np.all(np.diag(G) == n)             # C(t, t) = 1
        for k in range(K):
            assert full["bond"][r, k] == int(S[k, r] @ A @ S[k, r])
    for k in range(K):
        assert full["overlap"][0, k] == int(S[k, 0] @ S[k, 1])
    assert np.array_equal(S[-1], full["spins"].astype(np.int64))
    for r in range(2):
        init = np.array([oracle.init_spin(4, 6, r, i) for i in range(n)], np.int64)
        assert np.array_equal(S[0, r], init)
        assert full["gram"][r, 0, -1] == int(init @ S[-1, r])


def test_sk_infinite_temperature_observables_alternate():
    # T = inf: every move is accepted, s(t) = (-1)^t s(0), so the Gram matrix
    # is +-N by the parity of t - t', and bond sums and overlaps are constant.
    n = 300
    J = oracle.sk_couplings(n, seed=2, graph_id=5)
    o = oracle.sk_run(n, J, math.inf, 2, 1, 3, 64, 64)
    times = o["times"]
    for k, t in enumerate(times):
        for l, u in enumerate(times):
            assert np.all(o["gram"][:, k, l] == (n if (t - u) % 2 == 0 else -n))
    assert np.all(o["bond"] == o["bond"][:, :1])
    assert np.all(o["overlap"] == o["overlap"][:, :1])
    s0 = oracle.sk_run(n, J, math.inf, 2, 1, 3, 0, 64)["spins"].astype(np.int64)
    pairs = [(a, b) for a in range(3) for b in range(a + 1, 3)]
    for p, (a, b) in enumerate(pairs):
        assert o["overlap"][p, 0] == int(s0[a] @ s0[b])
