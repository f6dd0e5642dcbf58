"""Host logic of the serving loop (no GPU): batch selection by arrival,
(kind, run length) class (longest first), slot limit and HBM budget;
footprint bounds; VB contexts created in admission order."""
from paper_1906_11195_amd import serving, workloads


def R(rid, t, kind="vb", n=4096, sweeps=256):
    return workloads.Request(rid, t, kind, n, 0.7, sweeps)


def test_batch_takes_longest_class_first_in_arrival_order():
    pend = [R(0, 0.0, "sk"), R(1, 0.1), R(2, 0.2, "sk"), R(3, 0.3, "sk", sweeps=512), R(4, 5.0, "sk", sweeps=4096)]
    batch, fp = serving.select_batch(pend, now=1.0, time_scale=1.0, used=0, active_requests=0,
                                     budget=1 << 40, max_batch=8, max_active=64)
    assert [r.rid for r in batch] == [3]              # the longest class that has arrived by t = 1
    assert fp == serving.footprint_bytes("sk", 4096, 512)
    rest = [r for r in pend if r.rid != 3]
    batch, fp = serving.select_batch(rest, 1.0, 1.0, 0, 0, 1 << 40, 8, 64)
    assert [r.rid for r in batch] == [0, 2]           # same (kind, sweeps), in arrival order
    assert fp == sum(serving.footprint_bytes(r.kind, r.n, r.sweeps) for r in batch)
    # a class is as long as its longest run; equally long classes: the one that arrived first
    two = [R(0, 0.0, "vb", n=1000), R(1, 0.1, "vb", n=1000, sweeps=128), R(2, 0.2, "vb", n=4000, sweeps=128)]
    assert [r.rid for r in serving.select_batch(two, 1.0, 1.0, 0, 0, 1 << 40, 8, 64)[0]] == [1, 2]
    tie = [R(0, 0.0, "vb", n=2000), R(1, 0.1, "vb", n=4000, sweeps=128)]
    assert [r.rid for r in serving.select_batch(tie, 1.0, 1.0, 0, 0, 1 << 40, 8, 64)[0]] == [0]
    # one request at a time: arrival order
    assert serving.select_batch(pend, 0.05, 1.0, 0, 0, 1 << 40, 8, 64)[0][0].rid == 0


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


def test_vb_contexts_are_created_in_admission_order(monkeypatch):
    # worker threads that reach creation out of order still create their
    # contexts in ticket (admission) order; SK contexts do not take a turn
    import threading
    import time
    made = []
    monkeypatch.setattr(serving, "sg_create_vb",
                        lambda descs, t_max, split_members=0: made.append(("vb", descs[0].instance_id, split_members)) or "ctx")
    monkeypatch.setattr(serving, "sg_create_sk", lambda descs, t_max: made.append(("sk", descs[0].instance_id)) or "ctx")
    srv = serving.AgingServer.__new__(serving.AgingServer)
    srv._turn = threading.Condition()
    srv._tickets = 0
    srv._created = 0
    jobs = [([R(10 + t, 0.0)], t) for t in range(4)] + [([R(99, 0.0, "sk", n=512)], None), ([R(98, 0.0)], None)]
    threads = [threading.Thread(target=srv._create, args=job) for job in reversed(jobs)]
    for th in threads:
        th.start()
        time.sleep(0.01)
    for th in threads:
        th.join(timeout=10)
        assert not th.is_alive()
    # the batches that may split in ticket order; the short one (no ticket)
    # at once and with every unit whole
    assert [m for m in made if m[0] == "vb" and m[1] != 98] == [("vb", 10 + t, 0) for t in range(4)]
    assert made[:2] == [("vb", 98, 1), ("sk", 99)]
    assert srv._created == 4
