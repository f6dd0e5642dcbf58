"""Host logic of the serving loop (no GPU): batch selection by arrival,
(kind, run length) class, slot limit and HBM budget; footprint bounds."""
from paper_1906_11195_amd import serving, workloads


def R(rid, t, kind="vb", n=4096, sweeps=256):
    return workloads.Request(rid, t, kind, n, 0.7, sweeps)


def test_batch_takes_oldest_class_in_arrival_order():
    pend = [R(0, 0.0, "sk"), R(1, 0.1), R(2, 0.2, "sk"), R(3, 0.3, "sk", sweeps=512), R(4, 5.0, "sk")]
    batch, fp = serving.select_batch(pend, now=1.0, time_scale=1.0, used=0, active_requests=0,
                                     budget=1 << 40, max_batch=8, max_active=64)
    assert [r.rid for r in batch] == [0, 2]           # same (kind, sweeps), arrived by t = 1
    assert fp == sum(serving.footprint_bytes(r.kind, r.n, r.sweeps) for r in batch)


def test_batch_respects_limits():
    pend = [R(i, 0.0) for i in range(10)]
    b, _ = serving.select_batch(pend, 1.0, 1.0, 0, 0, 1 << 40, max_batch=3, max_active=64)
    assert len(b) == 3
    b, _ = serving.select_batch(pend, 1.0, 1.0, 0, 62, 1 << 40, max_batch=8, max_active=64)
    assert len(b) == 2
    one = serving.footprint_bytes("vb", 4096, 256)
    b, _ = serving.select_batch(pend, 1.0, 1.0, 0, 0, budget=int(2.5 * one), max_batch=8, max_active=64)
    assert len(b) == 2
    # nothing running: the first request is admitted even above the budget
    b, _ = serving.select_batch(pend, 1.0, 1.0, 0, 0, budget=1, max_batch=8, max_active=64)
    assert len(b) == 1
    b, _ = serving.select_batch(pend, 1.0, 1.0, 0, 1, budget=1, max_batch=8, max_active=64)
    assert b == []
    b, _ = serving.select_batch(pend, -1.0, 1.0, 0, 0, 1 << 40, 8, 64)
    assert b == []


def test_footprint_grows_with_size_and_length():
    assert serving.footprint_bytes("vb", 1 << 20, 4096) > serving.footprint_bytes("vb", 1 << 12, 4096)
    assert serving.footprint_bytes("sk", 8192, 4096) > 8192 * 8192          # the int8 couplings
    assert serving.footprint_bytes("vb", 4096, 1 << 16) > serving.footprint_bytes("vb", 4096, 1 << 8)
    assert serving.grid_len(1) == 2 and serving.grid_len(1024) == 12 and serving.grid_len(1023) == 11
