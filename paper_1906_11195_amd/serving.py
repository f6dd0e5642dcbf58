"""Continuous-batching request loop for aging runs on one GPU.

Requests (VB or SK aging runs of different sizes, temperatures and lengths)
arrive over time.  The server admits a request as soon as a slot is free and
its device-memory footprint fits the budget, keeps its spins on the device,
and advances every admitted run in chunks of sweeps on a pool of streams, so
that the runs of many requests are in flight on the device at once and a new
arrival does not wait for the others to finish.  A finished run is measured
(its observables copied to the host), its memory is released and the next
waiting request can take its place.

Every run is a pure function of its descriptor (counter-based random numbers
keyed by instance), so its result is the same alone and in any mix; the
serving test checks exactly that.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import (MEASURE_OBS, MEASURE_SPINS, SkDesc, VbDesc, sg_create_sk, sg_create_vb, sg_free,
               sg_measure, sg_sweep)


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


class AgingServer:
    def __init__(self, hbm_budget: int = 32 << 30, max_active: int = 64, chunk_sweeps: int = 256,
                 n_streams: int = 4, flags: int = MEASURE_OBS | MEASURE_SPINS):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.chunk = int(chunk_sweeps)
        self.flags = flags
        self.streams = [torch.cuda.Stream() for _ in range(max(1, n_streams))]

    def run(self, requests, time_scale: float = 1.0, max_wall: Optional[float] = None) -> List[Result]:
        """Serves `requests` (sorted by arrival time, seconds from the start,
        scaled by time_scale).  Returns one Result per finished request."""
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        active: Dict[int, dict] = {}
        used = 0
        results: List[Result] = []
        t0 = time.perf_counter()
        next_stream = 0
        while pending or active:
            now = time.perf_counter() - t0
            if max_wall is not None and now > max_wall:
                break
            # admission: arrived requests, free slot, footprint within budget
            while pending and pending[0].arrival * time_scale <= now and len(active) < self.max_active:
                req = pending[0]
                fp = footprint_bytes(req.kind, req.n, req.sweeps)
                if used + fp > self.budget and active:
                    break
                pending.pop(0)
                stream = self.streams[next_stream % len(self.streams)]
                next_stream += 1
                with torch.cuda.stream(stream):
                    d = descriptor(req)
                    ctx = (sg_create_vb if req.kind == "vb" else sg_create_sk)([d], t_max=req.sweeps)
                active[req.rid] = dict(req=req, ctx=ctx, stream=stream, done=0, event=None, fp=fp,
                                       admitted=time.perf_counter() - t0)
                used += fp
            progressed = False
            for rid in list(active):
                a = active[rid]
                ev = a["event"]
                if ev is not None and not ev.query():
                    continue
                req = a["req"]
                if a["done"] >= req.sweeps:
                    obs = sg_measure(a["ctx"], self.flags, stream=a["stream"])
                    sg_free(a["ctx"])
                    fin = time.perf_counter() - t0
                    results.append(Result(rid, req.kind, req.n, req.sweeps, req.arrival * time_scale,
                                          a["admitted"], fin, obs))
                    used -= a["fp"]
                    del active[rid]
                    progressed = True
                    continue
                k = min(self.chunk, req.sweeps - a["done"])
                sg_sweep(a["ctx"], k, stream=a["stream"])
                a["done"] += k
                ev = torch.cuda.Event()
                ev.record(a["stream"])
                a["event"] = ev
                progressed = True
            if not progressed:
                if active:
                    time.sleep(0.0002)
                elif pending:
                    wait = pending[0].arrival * time_scale - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
        for a in active.values():
            torch.cuda.synchronize()
            sg_free(a["ctx"])
        return results


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results]) if results else np.zeros(0)
    if lat.size == 0:
        return dict(count=0)
    return dict(count=int(lat.size), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3))
