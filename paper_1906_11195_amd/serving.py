"""Continuous-batching request loop for aging runs on one GPU.

Requests (VB or SK aging runs of different sizes, temperatures and lengths)
arrive over time.  The server admits a request as soon as a slot is free and
its device-memory footprint fits the budget, keeps its spins on the device,
and enqueues every admitted run's sweeps at admission on one of a pool of
streams, so that the runs of many requests are in flight on the device at
once and a new arrival does not wait for the others to finish.  A finished run is measured
(its observables copied to the host), its memory is released and the next
waiting request can take its place.

Every run is a pure function of its descriptor (counter-based random numbers
keyed by instance), so its result is the same alone and in any mix; the
serving test checks exactly that.
"""
from __future__ import annotations

import dataclasses
import os
import math
import threading
import time
from typing import Dict, List, Optional

import numpy as np

from . import (MEASURE_OBS, MEASURE_SPINS, SkDesc, VbDesc, sg_create_sk, sg_create_vb, sg_free,
               sg_measure, sg_sweep)


def hw_queues() -> int:
    """Hardware queues per process that HIP maps streams onto."""
    try:
        return max(1, int(os.environ.get("GPU_MAX_HW_QUEUES", "4")))
    except ValueError:
        return 4


def grid_len(t_max: int) -> int:
    return 2 + int(math.floor(math.log2(t_max))) if t_max >= 1 else 1


def footprint_bytes(kind: str, n: int, sweeps: int, replicas: int = 2, c: float = 4.0) -> int:
    """Upper bound of the device memory one run holds (the library's arena)."""
    K = grid_len(sweeps)
    wn = (n + 31) // 32
    chains = replicas
    common = chains * (K * wn * 4 + K * 8 + K * K * 8 + 8) + replicas * replicas * K * 8 + 64 * 1024
    if kind == "vb":
        m = int(c * n / 2)
        graph = 4 * (n + 1) + 8 * m + 4 * 64
        state = 4 * ((n * 8 + 31) // 32)
        units = 8 * 4608
        return int(1.1 * (graph + state + units + common)) + (1 << 20)
    J = n * n + n * wn * 4
    per_chain = chains * (wn * 4 + n * 4)
    thr = 8 * n
    return int(1.1 * (J + per_chain + thr + common)) + (1 << 20)


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    n: int
    sweeps: int
    arrival: float
    admitted: float
    finished: float
    obs: dict
    built: float = 0.0      # the batch's context built and all its sweeps enqueued (host)
    device: float = 0.0     # the batch's sweeps on its stream, first to last (HIP events)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def descriptor(req, seed: int = 5):
    if req.kind == "vb":
        return VbDesc(n=req.n, T=req.T, seed=seed, instance_id=req.rid, graph_id=req.rid, c=4.0,
                      n_replicas=2)
    return SkDesc(n=req.n, T=req.T, seed=seed, instance_id=req.rid, graph_id=req.rid, n_replicas=2)


def run_alone(req, flags: int = MEASURE_OBS | MEASURE_SPINS) -> dict:
    """The same run in a context of its own, start to finish."""
    d = descriptor(req)
    ctx = (sg_create_vb if req.kind == "vb" else sg_create_sk)([d], t_max=req.sweeps)
    try:
        sg_sweep(ctx, req.sweeps)
        return sg_measure(ctx, flags)
    finally:
        sg_free(ctx)


def estimate_device_s(kind: str, n: int, sweeps: int) -> float:
    """Coarse device time of one run with its chains whole (MI355X: a VB
    chain streams its graph at about 0.8 ns per spin and sweep; an SK chain
    takes about 100 us per sweep at N = 4096, growing as N^2).  Only used to
    order batches, longest first."""
    if kind == "vb":
        return sweeps * 0.8e-9 * n
    return sweeps * 100e-6 * (n / 4096.0) ** 2


def select_batch(pending, now: float, time_scale: float, used: int, active_requests: int, budget: int,
                 max_batch: int, max_active: int):
    """The next batch: of the requests that have arrived by `now`, the
    (kind, sweeps) class whose longest run takes longest on the device
    (longest first, so that a burst ends as early as it can; a class that
    arrived earlier wins ties, and requests arriving one at a time are taken
    in arrival order), its requests in arrival order as long as the batch
    stays within max_batch, the slot limit and the HBM budget (a batch always
    gets its first request when nothing else is running).  Returns (batch,
    its footprint in bytes)."""
    arrived = [r for r in pending if r.arrival * time_scale <= now]
    if not arrived:
        return [], 0
    longest: Dict[tuple, float] = {}
    for r in arrived:
        k = (r.kind, r.sweeps)
        longest[k] = max(longest.get(k, 0.0), estimate_device_s(r.kind, r.n, r.sweeps))
    key = max(longest, key=lambda k: longest[k])
    batch, fp_sum = [], 0
    for r in arrived:
        if (r.kind, r.sweeps) != key:
            continue
        if len(batch) >= max_batch or active_requests + len(batch) >= max_active:
            break
        fp = footprint_bytes(r.kind, r.n, r.sweeps)
        if used + fp_sum + fp > budget and (batch or active_requests):
            break
        batch.append(r)
        fp_sum += fp
    return batch, fp_sum


class AgingServer:
    """Continuous-batching loop over a pool of streams.

    A free stream takes every request that has arrived with the same kind and
    run length as the oldest waiting one (up to `max_batch`, within the HBM
    budget) and runs them as one context: all their chains advance in the same
    launches (large VB graphs split over several workgroups).  A batch's
    context is built on a worker thread (the host build releases the
    interpreter lock), and the worker enqueues all of the batch's sweeps on
    its stream (`chunk_sweeps` per call) at once, so the device never waits
    for the loop; new arrivals form the next batch on the next free stream
    while earlier ones run.  A batch is measured and released when its stream
    has finished; each request's result is its own slice of the batch's
    observables, identical to the run alone.

    Streams beyond the process's hardware queues (HIP's GPU_MAX_HW_QUEUES,
    4 unless set) share queues, and work on a shared queue runs in
    submission order: a batch whose sweeps are all enqueued at admission
    then holds back every batch queued behind it on the same queue.  So the
    pool defaults to one stream per hardware queue (n_streams = None), and a
    larger pool wants GPU_MAX_HW_QUEUES raised before the first HIP call.

    A VB batch whose longest run is estimated at `split_min_s` seconds or
    more may split its large graphs over several workgroups; such batches
    are created one at a time in admission order (the worker threads take
    turns): a context reserves the workgroups of its split units from a
    process-wide budget when it is created, so the batch admitted first, the
    longest, gets them first.  Shorter VB batches keep every unit whole
    (a split would save them little) and are created at once."""

    def __init__(self, hbm_budget: int = 32 << 30, max_active: int = 64, chunk_sweeps: int = 256,
                 n_streams: Optional[int] = None, flags: int = MEASURE_OBS | MEASURE_SPINS,
                 max_batch: int = 64, split_min_s: float = 0.25, streams=None):
        import torch
        if n_streams is None:
            n_streams = hw_queues()
        self.torch = torch
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.max_batch = int(max_batch)
        self.chunk = max(1, int(chunk_sweeps))
        self.flags = flags
        # a caller running several servers one after another can hand them
        # the same streams (each stream HIP has seen holds a hardware queue)
        self.streams = list(streams) if streams else [torch.cuda.Stream() for _ in range(max(1, n_streams))]
        self.split_min_s = float(split_min_s)
        self._turn = threading.Condition()
        self._tickets = 0      # VB batches admitted that may split
        self._created = 0      # of those, the ones whose context creation has ended

    def _take_batch(self, pending, now, time_scale, used, active_requests):
        return select_batch(pending, now, time_scale, used, active_requests, self.budget, self.max_batch,
                            self.max_active)

    def _create(self, batch, ticket):
        if batch[0].kind == "sk":
            return sg_create_sk([descriptor(r) for r in batch], t_max=batch[0].sweeps)
        if ticket is None:
            return sg_create_vb([descriptor(r) for r in batch], t_max=batch[0].sweeps, split_members=1)
        with self._turn:
            self._turn.wait_for(lambda: self._created == ticket)
        try:
            return sg_create_vb([descriptor(r) for r in batch], t_max=batch[0].sweeps)
        finally:
            with self._turn:
                self._created += 1
                self._turn.notify_all()

    def _start(self, batch, stream, ticket=None):
        """Worker: builds the batch's context (a VB batch that may split:
        when its turn `ticket` comes) and enqueues all its sweeps on
        `stream`; returns (context, start event, completion event, host time
        when everything was enqueued)."""
        torch = self.torch
        with torch.cuda.stream(stream):
            ctx = self._create(batch, ticket)
            try:
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
                done, length = 0, batch[0].sweeps
                while done < length:
                    k = min(self.chunk, length - done)
                    sg_sweep(ctx, k, stream=stream)
                    done += k
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(stream)
            except BaseException:
                sg_free(ctx)
                raise
        return ctx, ev0, ev, time.perf_counter()

    def run(self, requests, time_scale: float = 1.0, max_wall: Optional[float] = None) -> List[Result]:
        """Serves `requests` (arrival times in seconds from the start, scaled by
        time_scale).  Returns one Result per finished request."""
        from concurrent.futures import ThreadPoolExecutor
        pending = sorted(requests, key=lambda r: r.arrival)
        free = list(range(len(self.streams)))
        batches = []
        used = 0
        results: List[Result] = []
        pool = ThreadPoolExecutor(max_workers=len(self.streams))
        finisher = ThreadPoolExecutor(max_workers=len(self.streams))
        t0 = time.perf_counter()
        try:
            while pending or batches:
                now = time.perf_counter() - t0
                if max_wall is not None and now > max_wall:
                    break
                progressed = False
                # admission: a free stream takes the next batch
                while free and pending:
                    n_active = sum(len(b["reqs"]) for b in batches)
                    batch, fp = self._take_batch(pending, now, time_scale, used, n_active)
                    if not batch:
                        break
                    ids = set(id(r) for r in batch)
                    pending = [r for r in pending if id(r) not in ids]
                    si = free.pop(0)
                    ticket = None
                    if batch[0].kind == "vb" and max(estimate_device_s(r.kind, r.n, r.sweeps)
                                                     for r in batch) >= self.split_min_s:
                        ticket = self._tickets
                        self._tickets += 1
                    # the pool starts tasks in submission order, so a VB
                    # batch's turn never waits for one submitted after it
                    fut = pool.submit(self._start, batch, self.streams[si], ticket)
                    batches.append(dict(reqs=batch, fut=fut, si=si, fp=fp, admitted=now))
                    used += fp
                    progressed = True
                # completion: built, and its stream has run every sweep; the
                # batch is then measured and released on a worker thread, so
                # that a measurement waiting on its stream (a hardware queue
                # shared with another batch's sweeps) holds up no other batch
                for b in list(batches):
                    if "done" not in b:
                        if not b["fut"].done():
                            continue
                        ctx, ev0, ev, t_built = b["fut"].result()
                        if not ev.query():
                            continue
                        b["built"] = t_built - t0
                        b["done"] = finisher.submit(self._finish, ctx, ev0, ev, self.streams[b["si"]], t0)
                        progressed = True
                        continue
                    if not b["done"].done():
                        continue
                    obs, dev, fin = b["done"].result()
                    for i, req in enumerate(b["reqs"]):
                        results.append(Result(req.rid, req.kind, req.n, req.sweeps, req.arrival * time_scale,
                                              b["admitted"], fin, _slice(obs, i), built=b["built"], device=dev))
                    used -= b["fp"]
                    free.append(b["si"])
                    batches.remove(b)
                    progressed = True
                if not progressed:
                    if batches:
                        time.sleep(0.0002)
                    elif pending:
                        wait = pending[0].arrival * time_scale - (time.perf_counter() - t0)
                        if wait > 0:
                            time.sleep(min(wait, 0.01))
        finally:
            # release what is still in flight (after a time limit or an error)
            for b in batches:
                if "done" in b:
                    try:
                        b["done"].result()
                    except BaseException:
                        pass
                    continue
                try:
                    ctx, _, ev, _ = b["fut"].result()
                except BaseException:
                    continue
                ev.synchronize()
                sg_free(ctx)
            pool.shutdown(wait=True)
            finisher.shutdown(wait=True)
        return results

    def _finish(self, ctx, ev0, ev, stream, t0):
        """Worker: measures a finished batch on its stream and releases its
        context; returns (observables, device seconds, finish time)."""
        try:
            obs = sg_measure(ctx, self.flags, stream=stream)
        finally:
            sg_free(ctx)
        return obs, ev0.elapsed_time(ev) * 1e-3, time.perf_counter() - t0


def _slice(obs: dict, i: int) -> dict:
    """Instance i's observables, shaped like a one-instance context's."""
    out = {}
    for key, v in obs.items():
        if key in ("bond", "overlap", "gram", "accepted") and isinstance(v, np.ndarray):
            out[key] = v[i:i + 1]
        elif key == "spins" and v is not None:
            out[key] = [v[i]]
        else:
            out[key] = v
    return out


def latency_stats(results: List[Result]) -> dict:
    """p50 / p99 / mean latency, and where the mean goes: waiting for
    admission (arrival to admission), the host build and enqueue of the
    batch's context, the batch's sweeps on the device, and the rest (the
    stream busy with other work before the sweeps start, completion polling,
    measurement)."""
    lat = np.array([r.latency for r in results]) if results else np.zeros(0)
    if lat.size == 0:
        return dict(count=0)
    queue = np.array([r.admitted - r.arrival for r in results])
    build = np.array([max(0.0, r.built - r.admitted) for r in results])
    device = np.array([r.device for r in results])
    rest = lat - queue - build - device
    return dict(count=int(lat.size), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                mean_split_ms=dict(queue=float(queue.mean() * 1e3), build=float(build.mean() * 1e3),
                                   device=float(device.mean() * 1e3), rest=float(rest.mean() * 1e3)))
