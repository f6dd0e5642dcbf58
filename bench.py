"""Throughput benchmark of the aging Metropolis hot path on one MI355X.

Workload (one step = one pass of the whole path over the batch): the batched
Viana-Bray configuration -- 256 Erdos-Renyi graphs (N = 65536, mean degree 4,
+-1 couplings) x 3 temperatures {0.6, 0.8, 1.2} x 2 replicas = 1536 chains --
advanced by `--sweeps-per-step` Metropolis sweeps (snapshots at grid times on
the device), followed by the measurement (bond sums, overlaps, int8-MFMA Gram
matrices of all snapshots).  Inputs are synthetic and seeded; all state is in
HBM before the timed region starts.

Prints one JSON line: attempted single-spin updates per ns (the paper counts
spin updates), plus the roofline of the dominant kernel (the VB sweep),
secondary figures for the plain one-instance run and the SK configuration,
and the CPU oracle timed on the host's cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spin flips/ns at 1 GPU (VB, SK), batched vs plain; p50/p99 run latency"
HBM_PEAK_GBS = 8000.0
HBM_PEAK_BPS = HBM_PEAK_GBS * 1e9
MFMA_INT8_PEAK_OPS = 5.0e15   # dense int8 MFMA, MI355X
# VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def vb_bytes_per_sweep(descs, R, chains_per_unit):
    """Algorithmic bytes of one VB sweep, by the scope table's model: per
    chain-update (c w / 8 + o) / r + 1/4 B -- every work unit (r chains of one
    graph) streams the graph once (row starts o = 4 B per vertex, entries of
    w = 32 bits, c per vertex on average), and each chain-update reads and
    writes its own spin bit-packed (1/4 B).  In this design the spins never
    leave LDS during a launch, so the own-spin quarter byte is LDS traffic and
    the HBM counters see only the graph stream.  Units hold up to
    `chains_per_unit` chains of one graph."""
    graphs = {}
    for d in descs:
        key = (d.n, d.c, d.seed, d.graph_id, None if d.edges is None else id(d.edges))
        m = math.floor(d.c * d.n / 2) if d.edges is None else len(d.J)
        graphs.setdefault(key, [d.n, m, 0])
        graphs[key][2] += R
    total = 0.0
    for n, m, chains in graphs.values():
        units = math.ceil(chains / chains_per_unit)
        total += units * (4 * (n + 1) + 8 * m) + chains * n / 4.0
    return total


def vb_chains_per_unit(n, R):
    """Chains per work unit the library packs for one graph with R chains
    when LDS is the limit (the planner's rule: R chains in R-slot words if
    they fit in 159 KiB with up to 16 wavefronts, else fewer)."""
    per = R
    while per > 1:
        rpad = 1 if per <= 1 else 2 if per <= 2 else 4 if per <= 4 else 8
        sw = -(-n // (32 // rpad))
        lds = ((sw + 3) & ~3) * 4 + 8 * 128 * 4 + 64 + 16 + 68 * 4 + 64 + 32 * 8 * 4 + 16 * 1024
        if lds <= 160 * 1024 - 1024:
            break
        per -= 1
    return per


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    f = math.floor(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


PROFILE_VB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                          "vb_sweep_kernel_vb_batched_n65536.md")
VB_KERNEL_SOURCES = ("sg_vb.hip", "sg_vb_unit.h", "sg_philox.h")


def vb_kernel_digest() -> str:
    """First 16 hex digits of SHA-256 over the VB sweep kernel's sources."""
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1906_11195_amd", "csrc")
    for f in VB_KERNEL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_values(prefix: str):
    """The `prefix`* key: value lines of the committed VB profile, or None when
    the kernel sources have changed since its counters were taken."""
    try:
        with open(PROFILE_VB) as fh:
            kv = dict(line.split(": ", 1) for line in fh.read().splitlines()
                      if line.startswith(prefix) and ": " in line)
    except OSError:
        return None
    if kv.get(prefix + "kernel_digest", "").strip() != vb_kernel_digest():
        return None
    return kv


def profiled_traffic(sweeps_per_launch: float):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE passes
    (already scaled by the copy-kernel calibration), or None when the kernel
    sources have changed since the counters were taken."""
    kv = _profile_values("traffic_")
    if kv is None:
        return None
    fetch = float(kv["traffic_fetch_kib_per_sweep"]) * 1024.0 * sweeps_per_launch
    write = float(kv["traffic_write_kib_per_launch"]) * 1024.0
    return int(fetch + write)


def profiled_valu_per_update():
    """VALU wave-instructions per chain-update from the committed SQ_INSTS_VALU
    pass, or None when the kernel sources have changed since."""
    kv = _profile_values("issue_")
    return None if kv is None else float(kv["issue_valu_per_update"])


def run_vb_batched(args, torch, sg, workloads):
    descs = workloads.vb_batched()
    R = 2
    t_max = workloads.VB_BATCHED_SWEEPS
    log("creating VB batched context (%d instances, %d chains)" % (len(descs), len(descs) * R))
    ctx = sg.sg_create_vb(descs, t_max=t_max, chains_per_unit=args.chains_per_unit,
                          threads_per_unit=args.threads)
    stream = torch.cuda.current_stream()
    S = args.sweeps_per_step
    chains_per_unit = args.chains_per_unit or 6

    def step():
        sg.sg_sweep(ctx, S, stream)
        return sg.sg_measure(ctx, sg.MEASURE_OBS, stream)

    for w in range(args.warmup):
        step()
        log("warmup step %d done" % (w + 1))
    torch.cuda.synchronize()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    accepted0 = None
    for k in range(args.steps):
        ev0[k].record(stream)
        sg.sg_sweep(ctx, S, stream)
        ev1[k].record(stream)
        res = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)
        if accepted0 is None:
            accepted0 = res["accepted"].sum()
        log("step %d done" % (k + 1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sweep_ms = sum(a.elapsed_time(b) for a, b in zip(ev0, ev1))
    elapsed = t1 - t0
    n_total = sum(d.n for d in descs) * R
    updates = n_total * S * args.steps
    res = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)
    sg.sg_free(ctx)
    cap = max(1, min(4096, (1 << 36) // n_total))
    launches_per_step = math.ceil(S / cap)
    bytes_per_sweep = vb_bytes_per_sweep(descs, R, chains_per_unit)
    launch_ms = sweep_ms / (args.steps * launches_per_step)
    launch_bytes = bytes_per_sweep * S / launches_per_step
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    # the kernel's own ceiling: VALU issue (one wave64 instruction per SIMD
    # every 4 cycles), with the instructions per chain-update from the profile
    vpu = profiled_valu_per_update()
    valu_issue = None
    if vpu is not None:
        rate = n_total * S / launches_per_step / (launch_ms * 1e-3)
        valu_issue = dict(achieved=round(rate * vpu / 1e9, 1), peak=round(VALU_ISSUE_PEAK / 1e9, 1),
                          unit="G wave-instructions/s", frac=round(rate * vpu / VALU_ISSUE_PEAK, 4),
                          per_update=vpu)
    return dict(
        value=updates / (elapsed * 1e9), elapsed=elapsed, updates=updates,
        sweep_kernel_updates_per_ns=updates / (sweep_ms * 1e6),
        accepted_per_ns=float(res["accepted"].sum() - accepted0) / (elapsed * 1e9) if accepted0 is not None else None,
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4),
                      traffic=profiled_traffic(S / launches_per_step), traffic_unit="bytes per launch",
                      kernel="vb_sweep_kernel", launch_ms=round(launch_ms, 4),
                      bytes_per_launch=int(launch_bytes), bytes_per_update=round(bytes_per_sweep / n_total, 3),
                      valu_issue=valu_issue),
        ms_per_step=elapsed * 1e3 / args.steps, t_done=res["t_done"])


def run_vb_plain(args, torch, sg, workloads):
    """Plain one-instance run (1024 spins, 2 replicas, 4096 sweeps): run latency."""
    d = workloads.vb_plain()
    lat, parts = [], []
    for rep in range(args.plain_runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = sg.sg_create_vb(d, t_max=workloads.VB_PLAIN_SWEEPS)
        t1 = time.perf_counter()
        sg.sg_sweep(ctx, workloads.VB_PLAIN_SWEEPS)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sg.sg_measure(ctx, sg.MEASURE_OBS)
        sg.sg_free(ctx)
        t3 = time.perf_counter()
        lat.append(t3 - t0)
        parts.append((t1 - t0, t2 - t1, t3 - t2))
    upd = 1024 * 2 * workloads.VB_PLAIN_SWEEPS
    med = [percentile([p[i] for p in parts], 50) * 1e3 for i in range(3)]
    return dict(workload="VB plain: N=1024, 2 replicas, T=0.8, 4096 sweeps (create + sweeps + measure)",
                updates_per_ns=upd / (percentile(lat, 50) * 1e9),
                p50_ms=percentile(lat, 50) * 1e3, p99_ms=percentile(lat, 99) * 1e3, runs=len(lat),
                create_ms=round(med[0], 3), sweeps_ms=round(med[1], 3), measure_ms=round(med[2], 3))


def run_sk(args, torch, sg, workloads):
    descs = workloads.sk_batch()
    ctx = sg.sg_create_sk(descs, t_max=workloads.SK_SWEEPS)
    stream = torch.cuda.current_stream()
    sg.sg_sweep(ctx, 64, stream)          # warm-up window (includes one recompute)
    torch.cuda.synchronize()
    a0 = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)["accepted"].sum()
    t0 = time.perf_counter()
    sg.sg_sweep(ctx, args.sk_sweeps, stream)
    res = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sg.sg_free(ctx)
    n, reps, period = 4096, 2, descs[0].recompute_period
    upd = 64 * reps * n * args.sk_sweeps
    acc = float(res["accepted"].sum() - a0) / upd
    rate = upd / el
    # algorithmic HBM bytes per attempted update: one bit-packed coupling row
    # per accepted flip (a N / 8) plus the int8 J read by the exact recompute
    # once per sample and period (N^2 / (period N R)); int8 MFMA work of the
    # recompute: 2 N^2 R per sample and period (2 N / period per update)
    hbm = rate * (acc * n / 8 + n / (period * reps))
    mfma = rate * 2.0 * n / period
    return dict(workload="SK: 64 samples x 2 replicas, N=4096, T=0.5, sweeps 64..%d" % (64 + args.sk_sweeps),
                updates_per_ns=rate / 1e9, accepted_fraction=acc, sweeps=args.sk_sweeps,
                roofline={"bound": "latency", "hbm_GBps": round(hbm / 1e9, 1),
                          "hbm_frac": round(hbm / HBM_PEAK_BPS, 4),
                          "mfma_int8_TOPs": round(mfma / 1e12, 3),
                          "mfma_frac": round(mfma / MFMA_INT8_PEAK_OPS, 6)})


def run_sk_gauss(args, torch, sg, workloads):
    """SK with Gaussian couplings (Eq. 1, variance 1/N, float32 given by the
    input module): 64 samples x 2 replicas, N = 4096, T = 0.5, fields in
    double, recomputed every 64 sweeps; timed over sweeps 8..72 (one
    recomputation inside)."""
    t0 = time.perf_counter()
    descs, _ = workloads.sk_gaussian_batch()
    gen_s = time.perf_counter() - t0
    ctx = sg.sg_create_sk(descs, t_max=workloads.SK_SWEEPS)
    stream = torch.cuda.current_stream()
    sg.sg_sweep(ctx, 8, stream)
    torch.cuda.synchronize()
    a0 = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)["accepted"].sum()
    S = args.sk_gauss_sweeps
    t0 = time.perf_counter()
    sg.sg_sweep(ctx, S, stream)
    res = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sg.sg_free(ctx)
    n, reps = 4096, 2
    upd = len(descs) * reps * n * S
    acc = float(res["accepted"].sum() - a0) / upd
    rate = upd / el
    # bytes per attempted update: one float32 coupling row (4 N B) per
    # accepted flip, the block's 64 x 64 tile (4 x 64 B per spin), and the
    # direct recomputation (4 N^2 B per chain every 64 sweeps: 4 N / 64 B)
    bpu = acc * 4 * n + 4 * 64 + 4 * n / 64
    return dict(workload="SK Gaussian: 64 samples x 2 replicas, N=4096, J ~ N(0, 1/N) float32, fields in "
                         "double, T=0.5, sweeps 8..%d" % (8 + S),
                updates_per_ns=rate / 1e9, accepted_fraction=acc, generate_s=round(gen_s, 2),
                roofline=dict(bound="hbm", bytes_per_update=round(bpu, 1),
                              achieved=round(rate * bpu / 1e9, 1), unit="GB/s",
                              frac=round(rate * bpu / HBM_PEAK_BPS, 4)))


def run_uneven(args, torch, sg, workloads):
    """Uneven batch: 1024 VB instances, N log-uniform in [2^10, 2^20], 2 replicas,
    autotuned launch groups, graph-replayed sweep chunks; a steady window."""
    descs = workloads.vb_uneven()
    t0 = time.perf_counter()
    ctx = sg.sg_create_vb(descs, t_max=workloads.VB_UNEVEN_SWEEPS, autotune=True, graph=True)
    create_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    sg.sg_sweep(ctx, 16, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sg.sg_sweep(ctx, args.uneven_sweeps, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sg.sg_free(ctx)
    upd = sum(d.n for d in descs) * 2 * args.uneven_sweeps
    # every instance has its own graph: 2 chains per unit (1 for the graphs
    # whose two chains do not fit in one workgroup's LDS)
    byts = sum(vb_bytes_per_sweep([d], 2, vb_chains_per_unit(d.n, 2)) for d in descs) * args.uneven_sweeps
    dev_s = e0.elapsed_time(e1) * 1e-3
    return dict(workload="VB uneven: 1024 instances, N log-uniform in [2^10, 2^20], c=4, T in {0.6,0.8,1.0}, "
                         "2 replicas; sweeps 16..%d, autotuned, hipGraph" % (16 + args.uneven_sweeps),
                updates_per_ns=upd / (el * 1e9), create_s=round(create_s, 2),
                roofline=dict(bound="hbm", achieved=round(byts / dev_s / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(byts / dev_s / HBM_PEAK_BPS, 4), bytes_per_update=round(byts / upd, 3),
                              device_ms=round(dev_s * 1e3, 3)))


def run_rrbg(args, torch, sg, workloads):
    """The paper's graph ensemble: 256 random regular bipartite graphs of degree 4
    (N = 65536, +-1 couplings, explicit edge lists) x 3 temperatures x 2
    replicas, the temperatures of a graph sharing its arrays (one unit per
    graph, as in the batched leg)."""
    t0 = time.perf_counter()
    descs = workloads.vb_rrbg_batched()
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx = sg.sg_create_vb(descs, t_max=workloads.VB_BATCHED_SWEEPS)
    create_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    sg.sg_sweep(ctx, 64, stream)
    torch.cuda.synchronize()
    S = args.rrbg_sweeps
    t0 = time.perf_counter()
    sg.sg_sweep(ctx, S, stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)
    sg.sg_free(ctx)
    upd = sum(d.n for d in descs) * 2 * S
    byts = vb_bytes_per_sweep(descs, 2, 6) * S
    return dict(workload="VB RRBG: 256 random regular bipartite graphs (degree 4, N=65536, J=+-1) x "
                         "T{0.6,0.8,1.2} x 2 replicas; sweeps 64..%d" % (64 + S),
                updates_per_ns=upd / (el * 1e9), generate_s=round(gen_s, 2), create_s=round(create_s, 2),
                t_done=res["t_done"],
                roofline=dict(bound="hbm", frac=round(byts / el / HBM_PEAK_BPS, 4), unit="GB/s",
                              achieved=round(byts / el / 1e9, 1), bytes_per_update=round(byts / upd, 3)))


def run_multispin(args, torch, sg, workloads):
    """The paper's multispin workload (Methods; SI bipartite-graph section):
    256 random regular bipartite graphs (degree 4, N = 8192), 32 coupling
    samples x 2 replicas on each = 16384 chains, T cycling over {0.6, 0.8,
    1.2}.  Run in the multispin layout (64 chains of a graph per 64-bit word)
    and in the per-chain layout (each sample's two replicas share one unit),
    same sweeps, both timed."""
    t0 = time.perf_counter()
    descs = workloads.vb_multispin_batched()
    gen_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    S = args.multispin_sweeps
    out = dict(workload="VB multispin: 256 RRBG graphs (degree 4, N=8192) x 32 coupling samples x 2 replicas "
                        "= 16384 chains, T{0.6,0.8,1.2}; sweeps 16..%d" % (16 + S), generate_s=round(gen_s, 2))
    n_total = sum(d.n for d in descs) * 2
    res = {}
    for name, ms in (("multispin", True), ("per_chain", False)):
        t0 = time.perf_counter()
        ctx = sg.sg_create_vb(descs, t_max=workloads.VB_BATCHED_SWEEPS, multispin=ms)
        create_s = time.perf_counter() - t0
        sg.sg_sweep(ctx, 16, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        sg.sg_sweep(ctx, S, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)
        measure_ms = (time.perf_counter() - t0) * 1e3
        sg.sg_free(ctx)
        dev_s = e0.elapsed_time(e1) * 1e-3
        res[name] = r
        out[name] = dict(updates_per_ns=n_total * S / (el * 1e9), sweep_kernel_updates_per_ns=n_total * S / (dev_s * 1e9),
                         create_s=round(create_s, 2), measure_ms=round(measure_ms, 1))
    # bytes per chain-update by the scope table's model, r chains sharing the
    # graph stream, plus the per-chain couplings the multispin layout reads
    # with it (one bit per chain and adjacency entry: c / 8 B)
    bpu_ms = (4 * 4 + 4) / 64 + 0.25 + 4 / 8
    bpu_pc = (4 * 4 + 4) / 2 + 0.25
    for name, bpu in (("multispin", bpu_ms), ("per_chain", bpu_pc)):
        rate = out[name]["sweep_kernel_updates_per_ns"] * 1e9
        out[name]["roofline"] = dict(bound="hbm", bytes_per_update=round(bpu, 3), achieved=round(rate * bpu / 1e9, 1),
                                     unit="GB/s", frac=round(rate * bpu / HBM_PEAK_BPS, 4))
    out["identical"] = bool(all(np.array_equal(res["multispin"][k], res["per_chain"][k])
                                for k in ("bond", "gram", "accepted", "overlap")))
    out["speedup"] = round(out["multispin"]["updates_per_ns"] / out["per_chain"]["updates_per_ns"], 3)
    return out


def run_window(args, torch, sg, workloads):
    """The batched configuration with the paper's windowed estimator of C
    (SG_OPT_WINDOW, waiting times 0, 1, 2, 4, .., 2^12): after every sweep
    each chain's overlap with each of the 14 stored waiting-time
    configurations is added to its minor-third interval sum.  Timed past
    t = 2^12, where every waiting time contributes."""
    descs = workloads.vb_batched()
    R, tw_max = 2, 4096
    ctx = sg.sg_create_vb(descs, t_max=workloads.VB_BATCHED_SWEEPS, window_tw_max=tw_max)
    stream = torch.cuda.current_stream()
    sg.sg_sweep(ctx, tw_max + 1, stream)
    torch.cuda.synchronize()
    S = args.window_sweeps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sg.sg_sweep(ctx, S, stream)
    e1.record(stream)
    res = sg.sg_measure(ctx, sg.MEASURE_OBS, stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sg.sg_free(ctx)
    dev_s = e0.elapsed_time(e1) * 1e-3
    n_total = sum(d.n for d in descs) * R
    upd = n_total * S
    kw = res["window"].shape[2]
    # the sweep's own bytes plus the stored waiting-time words each unit reads
    # per sweep: kw x (8 slots x N / 8) B per 6-chain unit
    sweep_b = vb_bytes_per_sweep(descs, R, 6)
    win_b = 256 * kw * 65536 * 8 / 8
    byts = (sweep_b + win_b) * S
    return dict(workload="VB batched with the windowed C estimator (%d waiting times <= 2^12, minor-third "
                         "intervals of t_w + t): sweeps %d..%d" % (kw, tw_max + 1, tw_max + 1 + S),
                updates_per_ns=upd / (el * 1e9), sweep_kernel_updates_per_ns=upd / (dev_s * 1e9),
                roofline=dict(bound="hbm", achieved=round(byts / dev_s / 1e9, 1), peak=HBM_PEAK_GBS,
                              unit="GB/s", frac=round(byts / dev_s / HBM_PEAK_BPS, 4),
                              bytes_per_update=round(byts / upd, 3),
                              window_bytes_per_update=round(win_b / n_total, 3)))


_SERVE_STREAMS = []


def serve_streams(torch):
    """The serving legs' stream pool, shared by their servers: every stream
    HIP has seen keeps a hardware queue, and a process with more queues than
    the hardware schedules at once runs every kernel slower."""
    if not _SERVE_STREAMS:
        _SERVE_STREAMS.extend(torch.cuda.Stream() for _ in range(SERVE_STREAMS))
    return list(_SERVE_STREAMS)


def run_serving(args, torch, sg, workloads):
    """Serving: Poisson arrivals, 70% VB (N in [2^12, 2^20]) / 30% SK (N in
    [512, 8192]), T ~ U[0.5, 0.9]; run lengths reduced to 2^8..2^10 sweeps so
    that the leg fits the benchmark's time budget."""
    from paper_1906_11195_amd import serving
    reqs = workloads.serving_requests(args.serve_requests, rate=200.0)
    rng_len = [256, 512, 1024]
    for i, r in enumerate(reqs):
        r.sweeps = rng_len[i % 3]
    server = serving.AgingServer(hbm_budget=64 << 30, max_active=64, chunk_sweeps=256,
                                 streams=serve_streams(torch), flags=sg.MEASURE_OBS)
    t0 = time.perf_counter()
    results = server.run(reqs, max_wall=120.0)
    el = time.perf_counter() - t0
    st = serving.latency_stats(results)
    upd = sum(2 * r.n * r.sweeps for r in results)
    st.update(workload="serving: %d Poisson requests at 200/s, 70%% VB N in [2^12,2^20], 30%% SK N in "
                       "[512,8192], T~U[0.5,0.9], 256..1024 sweeps" % len(reqs),
              updates_per_ns=upd / (el * 1e9), wall_s=round(el, 2))
    return st


def served_bytes(results):
    """Algorithmic bytes of the served runs: VB by the scope table's model
    (one unit of the request's two chains streams its graph every sweep, two
    units of one chain each when two chains do not fit in LDS, plus 1/4 B per
    chain-update); SK by this library's model (one bit-packed coupling row of
    N / 8 B per accepted flip, plus the int8 couplings the exact recompute
    reads once per 64 sweeps for both chains)."""
    total = 0.0
    for r in results:
        if r.kind == "vb":
            units = 2 // vb_chains_per_unit(r.n, 2)
            total += r.sweeps * (units * (4 * (r.n + 1) + 8 * math.floor(2.0 * r.n)) + 2 * r.n / 4.0)
        else:
            acc = float(r.obs["accepted"].sum())
            total += acc * r.n / 8.0 + r.sweeps * r.n * r.n / 64.0
    return total


def run_serving_configured(args, torch, sg, workloads):
    """Serving at the configured run lengths: 2^k sweeps, k uniform in
    {12..16}, 70 % VB (N log-uniform in [2^12, 2^20]) and 30 % SK (N
    log-uniform in [512, 8192]), T ~ U[0.5, 0.9], 2 replicas.  The capacity is
    measured first, with every request arriving at once; the requests then
    arrive as a Poisson process at 0.8 x that capacity (the same requests,
    only the arrival times scaled)."""
    import dataclasses
    from paper_1906_11195_amd import serving
    n_req = args.serve_full_requests
    base = workloads.serving_requests(n_req, rate=1.0)

    def serve(reqs, max_wall):
        server = serving.AgingServer(hbm_budget=64 << 30, max_active=128, chunk_sweeps=4096,
                                     streams=serve_streams(torch), flags=sg.MEASURE_OBS)
        t0 = time.perf_counter()
        out = server.run(reqs, max_wall=max_wall)
        return out, time.perf_counter() - t0

    sat, w_sat = serve([dataclasses.replace(r, arrival=0.0) for r in base], args.serve_max_wall)
    log("serving capacity: %d requests in %.1f s" % (len(sat), w_sat))
    cap = len(sat) / w_sat
    rate = 0.8 * cap
    reqs = workloads.serving_requests(n_req, rate=rate)
    res, wall = serve(reqs, args.serve_max_wall)
    st = serving.latency_stats(res)
    upd = sum(2 * r.n * r.sweeps for r in res)
    byts = served_bytes(res)
    st.update(workload="serving at configured lengths: %d Poisson requests at 0.8 x measured capacity "
                       "(%.2f/s), 70%% VB N in [2^12,2^20], 30%% SK N in [512,8192], T~U[0.5,0.9], "
                       "2^12..2^16 sweeps" % (len(reqs), rate),
              capacity_per_s=round(cap, 3), capacity_wall_s=round(w_sat, 2), rate_per_s=round(rate, 3),
              served=len(res), updates_per_ns=upd / (wall * 1e9), wall_s=round(wall, 2),
              hbm=dict(achieved=round(byts / wall / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                       frac=round(byts / wall / HBM_PEAK_BPS, 4)),
              p50_by_kind_ms={k: float(np.percentile([r.latency for r in res if r.kind == k], 50) * 1e3)
                              for k in ("vb", "sk") if any(r.kind == k for r in res)})
    return st


def cpu_model() -> str:
    """The host CPU's model name (first `model name` line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(args, workloads):
    """The oracle, as it stands, on a bounded sample of the same workload:
    `threads` instances of the batched configuration (N = 65536, 2 replicas)
    for a few sweeps each, one instance per host thread."""
    import concurrent.futures as cf
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    # one oracle instance per core of this process's CPU share: the cores it
    # may run on, limited by the thread allotment the host sets for it
    # (OMP_NUM_THREADS), which is its share of a machine shared by several GPUs
    share = os.environ.get("OMP_NUM_THREADS", "")
    threads = max(1, min(cores, int(share))) if share.isdigit() and int(share) > 0 else max(1, cores)
    descs = workloads.vb_batched()[:threads]
    graphs = [oracle.vb_instance(d.n, d.c, d.seed, d.graph_id) for d in descs]
    # calibrate the cost of one sweep of one instance: the difference of a
    # 5-sweep and a 1-sweep run (each run also builds the instance's tables)
    eu, ev, J = graphs[0]
    cost = []
    for n_sw in (1, 5):
        t0 = time.perf_counter()
        oracle.vb_run(descs[0].n, eu, ev, J, descs[0].T, descs[0].seed, descs[0].instance_id, 2, n_sw, n_sw)
        cost.append(time.perf_counter() - t0)
    one = max((cost[1] - cost[0]) / 4.0, 1e-4)
    sweeps = int(max(2, min(4096, args.cpu_seconds / one)))

    def job(i):
        d = descs[i]
        eu, ev, J = graphs[i]
        oracle.vb_run(d.n, eu, ev, J, d.T, d.seed, d.instance_id, 2, sweeps, sweeps)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(job, range(threads)))
    el = time.perf_counter() - t0
    upd = threads * 2 * 65536 * sweeps
    return dict(value=upd / (el * 1e9), unit="attempted spin updates/ns", cores=threads, kind="oracle",
                host_cpus=cores, cpu_model=cpu_model(),
                sample="%d instances of the batched VB workload (N=65536, 2 replicas), %d sweeps each, "
                       "one instance per thread (%d host CPUs visible); %.1f s" % (threads, sweeps, cores, el))


# The serving legs keep a pool of SERVE_STREAMS streams.  Streams sharing a
# hardware queue run in submission order, so a batch would wait for every
# batch enqueued before it on its queue, and so would the measurement of a
# finished one; the library's own streams and the legacy stream take queues
# too.  So the serving legs run in a child process with SERVE_QUEUES hardware
# queues, twice the pool (16 streams on 16 queues: 1.3 s of the mean latency
# at configured lengths waited on shared queues; on 32: 3 ms), while the
# other legs keep MAIN_QUEUES (the uneven batch's launch groups on forked
# streams: 304-306 updates/ns on 8 queues, 287 on 32).  The number is set
# before HIP starts.
SERVE_STREAMS = 16
SERVE_QUEUES = 32
MAIN_QUEUES = 8


def run_serving_child(args, legs):
    """Runs the serving legs `legs` in a child process of this script with
    SERVE_QUEUES hardware queues; returns its (serving, serving_full) dicts."""
    import subprocess
    import torch
    torch.cuda.empty_cache()   # this process's cached blocks, for the child's use
    env = dict(os.environ, GPU_MAX_HW_QUEUES=str(SERVE_QUEUES))
    cmd = [sys.executable, os.path.abspath(__file__), "--serve-child", "--skip-headline", "--no-cpu-baseline",
           "--legs", ",".join(legs), "--serve-requests", str(args.serve_requests),
           "--serve-full-requests", str(args.serve_full_requests), "--serve-max-wall", str(args.serve_max_wall)]
    out = subprocess.run(cmd, env=env, stdout=subprocess.PIPE, text=True)
    if out.returncode != 0:
        # the other legs and the headline still run; the failure is reported
        # in place of the serving figures
        err = {"error": "serving legs failed in the child process (exit %d)" % out.returncode}
        log(err["error"])
        return (err if "serving" in legs else None), (err if "serving_full" in legs else None)
    d = json.loads(out.stdout.strip().splitlines()[-1])["legs"]
    return d.get("serving"), d.get("serving_full")


def main():
    child = "--serve-child" in sys.argv
    try:
        hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    except ValueError:
        hwq = 4
    want = SERVE_QUEUES if child else MAIN_QUEUES
    if hwq < want:
        os.environ["GPU_MAX_HW_QUEUES"] = str(want)
    ap = argparse.ArgumentParser()
    ap.add_argument("--serve-child", action="store_true",
                    help="internal: run the chosen serving legs in this process (the parent's child)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps-per-step", type=int, default=2048)
    ap.add_argument("--chains-per-unit", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--plain-runs", type=int, default=20)
    ap.add_argument("--sk-sweeps", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-vb", action="store_true", help="the batched VB leg only (same as --legs vb)")
    ap.add_argument("--legs", default="vb,plain,sk,sk_gauss,uneven,rrbg,multispin,window,serving,serving_full",
                    help="comma-separated legs to run besides the headline: plain, sk, sk_gauss, uneven, "
                         "rrbg, multispin, window, serving, serving_full")
    ap.add_argument("--multispin-sweeps", type=int, default=256)
    ap.add_argument("--sk-gauss-sweeps", type=int, default=64)
    ap.add_argument("--skip-headline", action="store_true",
                    help="run only the chosen legs (for profiling one leg; no headline value)")
    ap.add_argument("--uneven-sweeps", type=int, default=128)
    ap.add_argument("--rrbg-sweeps", type=int, default=512)
    ap.add_argument("--window-sweeps", type=int, default=512)
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-full-requests", type=int, default=96)
    ap.add_argument("--serve-max-wall", type=float, default=120.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(batches would shard by instance with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1906_11195_amd as sg
    from paper_1906_11195_amd import workloads

    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        # A plain copy kernel of known size: reads and writes exactly
        # copy_probe_mib MiB; used to scale the FETCH_SIZE / WRITE_SIZE counters.
        n = args.copy_probe_mib << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            # evict the source from the caches (L2 and the 256 MB Infinity
            # Cache) with an unrelated fill before each copy
            evict = torch.full((512 << 20,), 3, dtype=torch.uint8, device="cuda")
            del evict
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "launches": 3}), flush=True)
        return
    sg.library()
    legs = set() if args.only_vb else set(x.strip() for x in args.legs.split(","))
    # the serving legs run first, in a child process, while this process
    # holds next to no hardware queues (the queues of all processes on the
    # device share the hardware's scheduler: with this process's queues of
    # the other legs beside the child's, the capacity run took 29-31 s
    # instead of 21)
    serve = serve_full = None
    serve_legs = [x for x in ("serving", "serving_full") if x in legs]
    if serve_legs and not args.serve_child:
        serve, serve_full = run_serving_child(args, serve_legs)
    vb = None
    if not args.skip_headline:
        vb = run_vb_batched(args, torch, sg, workloads)
        log("VB batched: %.1f updates/ns" % vb["value"])
    plain = sk = uneven = rrbg = window = sk_gauss = multispin = None
    if "plain" in legs:
        plain = run_vb_plain(args, torch, sg, workloads)
        log("VB plain: p50 %.2f ms" % plain["p50_ms"])
    if "sk" in legs:
        sk = run_sk(args, torch, sg, workloads)
        log("SK: %.2f updates/ns" % sk["updates_per_ns"])
    if "sk_gauss" in legs:
        sk_gauss = run_sk_gauss(args, torch, sg, workloads)
        log("SK Gaussian: %.3f updates/ns" % sk_gauss["updates_per_ns"])
    if "uneven" in legs:
        uneven = run_uneven(args, torch, sg, workloads)
        log("VB uneven: %.1f updates/ns" % uneven["updates_per_ns"])
    if "rrbg" in legs:
        rrbg = run_rrbg(args, torch, sg, workloads)
        log("VB RRBG: %.1f updates/ns" % rrbg["updates_per_ns"])
    if "multispin" in legs:
        multispin = run_multispin(args, torch, sg, workloads)
        log("VB multispin: %.1f updates/ns (per-chain layout %.1f)" % (multispin["multispin"]["updates_per_ns"],
                                                                        multispin["per_chain"]["updates_per_ns"]))
    if "window" in legs:
        window = run_window(args, torch, sg, workloads)
        log("VB windowed C: %.1f updates/ns" % window["updates_per_ns"])
    if args.serve_child:
        if "serving" in legs:
            serve = run_serving(args, torch, sg, workloads)
            log("serving: p50 %.1f ms, p99 %.1f ms" % (serve.get("p50_ms", 0), serve.get("p99_ms", 0)))
        if "serving_full" in legs:
            serve_full = run_serving_configured(args, torch, sg, workloads)
            log("serving (configured lengths): p50 %.1f ms, p99 %.1f ms, %.1f updates/ns"
                % (serve_full.get("p50_ms", 0), serve_full.get("p99_ms", 0), serve_full["updates_per_ns"]))
    if vb is None:
        print(json.dumps({"legs": dict(plain=plain, sk=sk, sk_gauss=sk_gauss, uneven=uneven, rrbg=rrbg,
                                       multispin=multispin, window=window,
                                       serving=serve, serving_full=serve_full)}), flush=True)
        return
    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(args, workloads)
        log("cpu oracle: %.4f updates/ns on %d threads" % (cpu["value"], cpu["cores"]))

    out = {
        "metric": METRIC,
        "value": round(vb["value"], 3),
        "unit": "attempted spin updates/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(vb["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "VB batched: 256 ER graphs (N=65536, c=4, J=+-1) x T{0.6,0.8,1.2} x 2 replicas "
                        "= 1536 chains; step = %d sweeps + observables + int8-MFMA Gram" % args.sweeps_per_step,
            "sweeps_per_step": args.sweeps_per_step,
            "chains": 1536,
            "spins_per_chain": 65536,
            "parallelism": "1 GPU, one workgroup per graph (chains sharing its stream)",
        },
        "accepted_flips_per_ns": vb["accepted_per_ns"],
        "sweep_kernel_updates_per_ns": round(vb["sweep_kernel_updates_per_ns"], 3),
        "roofline": vb["roofline"],
        "cpu_baseline": cpu,
        "plain": plain,
        "sk": sk,
        "sk_gauss": sk_gauss,
        "uneven": uneven,
        "rrbg": rrbg,
        "multispin": multispin,
        "window": window,
        "serving": serve,
        "serving_configured": serve_full,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
