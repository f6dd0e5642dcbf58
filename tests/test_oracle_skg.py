"""CPU pins of the oracle's SK dynamics with real (Gaussian) couplings
(orc_skg_run; Eq. 1 with J_ij ~ N(0, 1/N)), against facts that do not come
from the oracle itself: the binary oracle (already pinned) when the real
couplings are +-1/sqrt(N) with 1/sqrt(N) exact in float32, the exact
master-equation transient and the Boltzmann stationary law of tiny systems
(tests/brute.py, closed-form Metropolis probabilities), T = inf and T = 0
limits, gauge and global-flip symmetry (bit for bit), the paramagnetic
energy, and observables recomputed from re-run configurations."""
import math

import numpy as np
import pytest

import oracle
from paper_1906_11195_amd.workloads import gaussian_couplings
from tests import brute


def bond_real(S, J):
    """B(s) = sum_{i<j} J_ij s_i s_j for every row of S (float64)."""
    return np.einsum("si,ij,sj->s", S.astype(float), J.astype(float), S.astype(float)) / 2.0


@pytest.mark.parametrize("n", [64, 256])
def test_binary_couplings_reproduce_the_binary_oracle(n):
    # 1/sqrt(N) = 2^-3 or 2^-4 is exact in float32, every field is then an
    # exact dyadic multiple of the integer field, and the acceptance
    # expression is the binary one term for term
    Jb = oracle.sk_couplings(n, seed=3, graph_id=5)
    Jr = (Jb.astype(np.float32) / np.float32(math.sqrt(n))).astype(np.float32)
    for T in (0.5, 1.3):
        a = oracle.sk_run(n, Jb, T, 3, 9, 2, 70, 64)
        b = oracle.skg_run(n, Jr, T, 3, 9, 2, 70, 64, period=16)
        assert np.array_equal(a["spins"], b["spins"])
        assert np.array_equal(a["accepted"], b["accepted"])
        assert np.array_equal(a["gram"], b["gram"]) and np.array_equal(a["overlap"], b["overlap"])
        assert np.allclose(b["bond"], a["bond"] / math.sqrt(n), rtol=0, atol=1e-12)


@pytest.mark.parametrize("T", [0.7, 2.0])
def test_transient_energy_matches_master_equation(T):
    n = 7
    J = gaussian_couplings(n, seed=11)
    S = brute.states(n)
    B = bond_real(S, J)
    n_inst, t_max = 6000, 8
    bonds = np.array([oracle.skg_run(n, J, T, 17, inst, 1, t_max, t_max)["bond"][0]
                      for inst in range(n_inst)], float)
    dist = np.full(1 << n, 1.0 / (1 << n))
    A = J.astype(float)
    t_now = 0
    for k, t in enumerate(oracle.grid(t_max)):
        while t_now < t:
            dist = brute.sweep(dist, S, A, list(range(n)), T, 1.0)
            t_now += 1
        m = float(dist @ B)
        se = math.sqrt(max(float(dist @ (B - m) ** 2), 1e-12) / n_inst)
        assert abs(bonds[:, k].mean() - m) < 5 * se, (t, bonds[:, k].mean(), m)


def test_one_sweep_operator_keeps_boltzmann_and_chains_reach_it():
    n, T = 5, 0.8
    J = gaussian_couplings(n, seed=4)
    S = brute.states(n)
    B = bond_real(S, J)
    w = np.exp((B - B.max()) / T)
    pi = w / w.sum()
    # the sweep operator of the closed-form probabilities leaves pi invariant
    assert np.abs(brute.sweep(pi, S, J.astype(float), list(range(n)), T, 1.0) - pi).max() < 1e-12
    # and independent chains sample it (final states after 64 sweeps)
    counts = np.zeros(1 << n)
    n_inst = 4000
    for inst in range(n_inst):
        s = oracle.skg_run(n, J, T, 5, inst, 1, 64, 64)["spins"][0]
        counts[int(sum(1 << i for i in range(n) if s[i] < 0))] += 1
    exp = pi * n_inst
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 80.0, chi2      # 31 degrees of freedom: p ~ 1e-6 at 80


def test_infinite_and_zero_temperature():
    n = 200
    J = gaussian_couplings(n, seed=2)
    rng = np.random.default_rng(1)
    s0 = rng.choice([-1, 1], size=(2, n)).astype(np.int8)
    c = oracle.skg_run(n, J, math.inf, 1, 4, 2, 9, 16, start=oracle.START_GIVEN, s0=s0)
    assert np.array_equal(c["spins"], -s0) and np.all(c["accepted"] == 9 * n)
    assert np.allclose(c["bond"][:, :c["k_done"]], c["bond"][:, :1], rtol=0, atol=1e-9)
    # T = 0: the energy -B never rises from one sweep to the next
    prev = None
    for t in range(0, 12):
        s = oracle.skg_run(n, J, 0.0, 1, 4, 1, t, 16)["spins"][0]
        b = float(bond_real(s[None, :], J)[0])
        if prev is not None:
            assert b >= prev - 1e-9
        prev = b


def test_gauge_and_global_flip_bit_for_bit():
    n, T = 160, 0.6
    J = gaussian_couplings(n, seed=6)
    rng = np.random.default_rng(3)
    s0 = rng.choice([-1, 1], size=(2, n)).astype(np.int8)
    g = rng.choice([-1, 1], size=n).astype(np.int8)
    a = oracle.skg_run(n, J, T, 1, 4, 2, 80, 64, period=32, start=oracle.START_GIVEN, s0=s0)
    Jg = (J * g[:, None].astype(np.float32) * g[None, :].astype(np.float32)).astype(np.float32)
    b = oracle.skg_run(n, Jg, T, 1, 4, 2, 80, 64, period=32, start=oracle.START_GIVEN,
                       s0=(s0 * g).astype(np.int8))
    assert np.array_equal(b["spins"], a["spins"] * g)
    assert np.array_equal(a["bond"], b["bond"]) and np.array_equal(a["gram"], b["gram"])
    assert np.array_equal(b["fields"], a["fields"] * g)
    f = oracle.skg_run(n, J, T, 1, 4, 2, 80, 64, period=32, start=oracle.START_GIVEN,
                       s0=(-s0).astype(np.int8))
    assert np.array_equal(f["spins"], -a["spins"]) and np.array_equal(f["bond"], a["bond"])


def test_incremental_fields_track_the_direct_sums():
    n, T = 300, 0.5
    J = gaussian_couplings(n, seed=8)
    a = oracle.skg_run(n, J, T, 2, 1, 2, 50, 64, period=0)        # never recomputed
    b = oracle.skg_run(n, J, T, 2, 1, 2, 50, 64, direct=True)
    c = oracle.skg_run(n, J, T, 2, 1, 2, 50, 64, period=7)
    for o in (a, c):
        assert np.array_equal(o["spins"], b["spins"]) and np.array_equal(o["accepted"], b["accepted"])
        assert np.abs(o["fields"] - b["fields"]).max() < 1e-12
    # the direct fields are J s of the final configuration
    s = b["spins"].astype(float)
    assert np.abs(b["fields"] - s @ J.astype(float).T).max() < 1e-12


def test_observables_recomputed_from_configurations():
    n, T, t_max = 120, 0.5, 32
    J = gaussian_couplings(n, seed=9)
    o = oracle.skg_run(n, J, T, 3, 2, 3, t_max, t_max, period=8)
    times = oracle.grid(t_max)
    snaps = np.array([[oracle.skg_run(n, J, T, 3, 2, 3, int(t), t_max, period=8)["spins"][r] for t in times]
                      for r in range(3)], np.int64)                 # [R][K][n]
    for r in range(3):
        assert np.array_equal(o["gram"][r], snaps[r] @ snaps[r].T)
        assert np.allclose(o["bond"][r], bond_real(snaps[r], J), rtol=0, atol=1e-9)
    pairs = [(0, 1), (0, 2), (1, 2)]
    for p, (a, b) in enumerate(pairs):
        assert np.array_equal(o["overlap"][p], (snaps[a] * snaps[b]).sum(1))
    assert np.all(np.diagonal(o["gram"], axis1=1, axis2=2) == n)


def test_paramagnet_energy_closed_form():
    # T > 1: e = -beta (N - 1) / (2 N) at leading order (annealed = quenched)
    n, T = 512, 2.0
    vals = []
    for smp in range(4):
        J = gaussian_couplings(n, seed=100 + smp)
        o = oracle.skg_run(n, J, T, 8, smp, 2, 96, 96)
        vals.extend((-o["bond"][:, -2:] / n).ravel())
    assert abs(np.mean(vals) - (-(1 / T) * (n - 1) / (2 * n))) < 0.02
