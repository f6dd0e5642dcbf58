"""Pins for the oracle's Philox generator and its stream layout (CPU only)."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_philox4x32_known_answers(ctr, key, want):
    assert list(oracle.philox4x32(ctr, key)) == want


@pytest.mark.parametrize("ctr0,key", [(0, (0, 0)), (5, (7, 9)), (2**40 + 3, (2**63 + 11, 12345)),
                                      (2**64 - 7, (1, 2**64 - 1))])
def test_philox4x64_matches_numpy(ctr0, key):
    # numpy's Philox is the 4x64-10 member of the same family, an independent
    # implementation; it advances the counter once before its first block.
    bg = np.random.Philox(counter=np.array([ctr0 % 2**64, 0, 0, 0], dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    raw = bg.random_raw(12)
    for blk in range(3):
        c = ctr0 + 1 + blk
        ctr = [c % 2**64, c // 2**64, 0, 0]
        got = oracle.philox4x64(ctr, key)
        assert [int(x) for x in got] == [int(x) for x in raw[4 * blk:4 * blk + 4]]


def test_accept_uniform_is_uniform_and_uncorrelated():
    # 64k draws over positions and sweeps: top-byte histogram (chi^2) and
    # lag-1 correlation between neighbouring positions.
    from scipy import stats
    seed, inst, rep = 12345, 3, 1
    r = np.array([oracle.accept_uniform(seed, inst, rep, t, p)
                  for t in range(16) for p in range(4096)], dtype=np.float64)
    hist = np.bincount((r.astype(np.uint64) >> np.uint64(24)).astype(np.int64), minlength=256)
    chi2, pval = stats.chisquare(hist)
    assert pval > 1e-4
    u = r / 2**32
    assert abs(u.mean() - 0.5) < 5 * (1 / np.sqrt(12 * len(u)))
    c = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(c) < 5 / np.sqrt(len(u))


def test_accept_uniform_halves_come_from_distinct_streams():
    # The high and low 16 bits must not be the same half-word.
    hi = [oracle.accept_uniform(1, 0, 0, 0, p) >> 16 for p in range(64)]
    lo = [oracle.accept_uniform(1, 0, 0, 0, p) & 0xFFFF for p in range(64)]
    assert hi != lo


def test_streams_depend_on_every_key_field():
    base = oracle.accept_uniform(7, 1, 0, 5, 100)
    assert oracle.accept_uniform(8, 1, 0, 5, 100) != base          # seed
    assert oracle.accept_uniform(7, 2, 0, 5, 100) != base          # instance
    assert oracle.accept_uniform(7, 1, 1, 5, 100) != base          # replica
    assert oracle.accept_uniform(7, 1, 0, 6, 100) != base          # sweep
    assert oracle.accept_uniform(7, 1, 0, 5, 101) != base          # position


def test_init_spins_are_balanced():
    s = np.array([oracle.init_spin(1, 0, 0, p) for p in range(1 << 15)])
    assert set(np.unique(s)) == {-1, 1}
    assert abs(s.sum()) < 5 * np.sqrt(len(s))
    s1 = np.array([oracle.init_spin(1, 0, 1, p) for p in range(1 << 12)])
    assert not np.array_equal(s[:1 << 12], s1)
