"""Seeded synthetic workloads (descriptor recipes only).

This module holds no arithmetic of the method: it only lists instance
descriptors (sizes, temperatures, seeds, ids) for the configurations the
benchmark and the tests run.  The paper's own graphs, couplings and data are
not available; these synthetic instances stand in for its workloads (random
regular bipartite graphs of degree 4 with +-1 couplings and binary SK
couplings, SI sections on the SK model and on the bipartite graph).

  VB plain    1 instance, 2 replicas, N = 1024, Erdos-Renyi c = 4, J = +-1,
              T = 0.8, random start, 4096 sweeps, grid {0} U {2^k}, seed 1.
  VB batched  256 graphs x T in {0.6, 0.8, 1.2} x 2 replicas (1536 chains),
              N = 65536, c = 4, 2^20 sweeps, seed 2; instance 3 s + tau on
              graph s.
  SK          64 samples x 2 replicas, N = 4096, binary couplings, T = 0.5,
              2^16 sweeps, fields recomputed every 64 sweeps, seed 3.
  VB uneven   1024 instances, N = floor(2^(10 + 10 U)), T from {0.6, 0.8, 1.0},
              2 replicas, 2^14 sweeps, seed 4 (U, T index from numpy's
              default_rng(4)).
  serving     Poisson arrivals; 70 % VB with N log-uniform in [2^12, 2^20],
              30 % SK with N log-uniform in [512, 8192]; T ~ U[0.5, 0.9];
              2^k sweeps, k uniform in {12..16}; seed 5.
  VB multispin  256 random regular bipartite graphs (degree 4, N = 8192),
              each with 32 coupling samples x 2 replicas (16384 chains), seed 8.
  VB RRBG     the paper's graph ensemble (SI, bipartite-graph section): 256
              random regular bipartite graphs of degree 4, N = 65536, +-1
              couplings, x T in {0.6, 0.8, 1.2} x 2 replicas, seed 6; the
              three temperatures of a graph pass the same edge arrays.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import VbDesc, SkDesc

VB_PLAIN_SWEEPS = 4096
VB_BATCHED_SWEEPS = 1 << 20
SK_SWEEPS = 1 << 16
VB_UNEVEN_SWEEPS = 1 << 14


def vb_plain() -> List[VbDesc]:
    return [VbDesc(n=1024, T=0.8, seed=1, instance_id=0, graph_id=0, c=4.0, n_replicas=2)]


def vb_batched(n_graphs: int = 256, n: int = 65536, temps=(0.6, 0.8, 1.2)) -> List[VbDesc]:
    out = []
    for s in range(n_graphs):
        for tau, T in enumerate(temps):
            out.append(VbDesc(n=n, T=T, seed=2, instance_id=len(temps) * s + tau, graph_id=s, c=4.0,
                              n_replicas=2))
    return out


def sk_batch(n_samples: int = 64, n: int = 4096, T: float = 0.5) -> List[SkDesc]:
    return [SkDesc(n=n, T=T, seed=3, instance_id=s, graph_id=s, n_replicas=2, recompute_period=64)
            for s in range(n_samples)]


def vb_uneven(count: int = 1024, lo: int = 10, hi: int = 20, temps=(0.6, 0.8, 1.0)) -> List[VbDesc]:
    rng = np.random.default_rng(4)
    U = rng.random(count)
    V = rng.random(count)
    out = []
    for i in range(count):
        n = int(np.floor(2.0 ** (lo + (hi - lo) * U[i])))
        T = temps[int(np.floor(len(temps) * V[i]))]
        out.append(VbDesc(n=n, T=T, seed=4, instance_id=i, graph_id=i, c=4.0, n_replicas=2))
    return out


def gaussian_couplings(n: int, seed: int) -> np.ndarray:
    """SK couplings of the main text (Eq. 1): J_ij = J_ji Gaussian with mean 0
    and variance 1/N, J_ii = 0, as float32 [n, n]: numpy default_rng(seed)
    float32 standard normals (row by row; the upper triangle is used) times
    float32(1 / sqrt(N)), mirrored to the lower triangle."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n), dtype=np.float32)
    J = np.triu(z, 1)
    J *= np.float32(1.0 / np.sqrt(float(n)))
    J += J.T
    return J


def sk_gaussian_batch(n_samples: int = 64, n: int = 4096, T: float = 0.5, seed: int = 7):
    """SK with Gaussian couplings: (descriptors, coupling matrices), one matrix
    per sample, 2 replicas each."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        Js = list(ex.map(lambda s: gaussian_couplings(n, seed * 1000003 + s), range(n_samples)))
    descs = [SkDesc(n=n, T=T, seed=seed, instance_id=s, graph_id=s, n_replicas=2, recompute_period=64,
                    Jf=Js[s]) for s in range(n_samples)]
    return descs, Js


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float       # seconds after the start
    kind: str            # "vb" or "sk"
    n: int
    T: float
    sweeps: int


def serving_requests(count: int, rate: float, seed: int = 5) -> List[Request]:
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        kind = "vb" if rng.random() < 0.7 else "sk"
        if kind == "vb":
            n = int(np.floor(2.0 ** rng.uniform(12, 20)))
        else:
            n = int(np.floor(2.0 ** rng.uniform(9, 13)))
        T = float(rng.uniform(0.5, 0.9))
        sweeps = 1 << int(rng.integers(12, 17))
        out.append(Request(rid, t, kind, n, T, sweeps))
    return out


def random_regular_edges(n: int, z: int, seed: int, bipartite: bool = False):
    """Edge list and +-1 couplings of a random z-regular graph on n vertices
    (bipartite: every edge joins {0 .. n/2 - 1} to {n/2 .. n - 1}).  The
    configuration model pairs the z stubs of every vertex at random (for the
    bipartite graph, the stubs of one half with those of the other); each
    self-loop or repeated edge is then removed by exchanging an endpoint with
    a randomly chosen other edge, which keeps every degree and the
    bipartition (a small dense graph whose repair stalls is paired again).
    Returns (int32 [m, 2], int8 [m]) with m = n z / 2."""
    if z < 1 or (z > n // 2 if bipartite else z >= n):
        raise ValueError("no simple %d-regular %sgraph on %d vertices" % (z, "bipartite " if bipartite else "", n))
    rng = np.random.default_rng(seed)
    if bipartite and n % 2:
        raise ValueError("bipartite graph needs an even n")
    if not bipartite and (n * z) % 2:
        raise ValueError("n z must be even")

    def code(u, v):
        return np.minimum(u, v) * n + np.maximum(u, v)

    def attempt():
        # one pairing and its repair; None when an exchange cannot be found
        # (small dense graphs), and the pairing is drawn again
        if bipartite:
            h = n // 2
            a = rng.permutation(np.repeat(np.arange(h, dtype=np.int64), z))
            b = rng.permutation(np.repeat(np.arange(h, n, dtype=np.int64), z))
            e = np.stack([a, b], axis=1)
        else:
            e = rng.permutation(np.repeat(np.arange(n, dtype=np.int64), z)).reshape(-1, 2)
        m = len(e)
        codes = code(e[:, 0], e[:, 1])
        _, first = np.unique(codes, return_index=True)
        bad = np.ones(m, bool)
        bad[first] = False
        bad |= e[:, 0] == e[:, 1]
        seen = {}
        for k, cd in enumerate(codes.tolist()):
            if not bad[k]:
                seen[cd] = k
        for i in np.flatnonzero(bad).tolist():
            for _ in range(4096):
                j = int(rng.integers(m))
                if j == i or bad[j]:
                    continue
                u, v = int(e[i, 0]), int(e[i, 1])
                x, y = int(e[j, 0]), int(e[j, 1])
                # (u, v), (x, y) -> (u, y), (x, v): degrees and halves unchanged
                c1, c2 = int(code(u, y)), int(code(x, v))
                if u == y or x == v or c1 == c2 or c1 in seen or c2 in seen:
                    continue
                del seen[int(codes[j])]
                e[i, 1], e[j, 1] = y, v
                codes[i], codes[j] = c1, c2
                seen[c1], seen[c2] = i, j
                bad[i] = False
                break
            else:
                return None
        return e

    for _ in range(10000):
        e = attempt()
        if e is not None:
            break
    else:
        raise RuntimeError("no simple %d-regular graph found on %d vertices" % (z, n))
    m = len(e)
    J = np.where(rng.random(m) < 0.5, -1, 1).astype(np.int8)
    return e.astype(np.int32), J


def vb_multispin_batched(n_graphs: int = 256, n: int = 8192, samples: int = 32, z: int = 4,
                         temps=(0.6, 0.8, 1.2), seed: int = 8) -> List[VbDesc]:
    """The paper's multispin workload shape (Methods; SI bipartite-graph
    section): random regular bipartite graphs of degree z, each carrying
    `samples` independent +-1 coupling sets (numpy default_rng(seed * 1000003
    + graph)), 2 replicas per sample, temperatures cycling over `temps`; 256 x
    32 x 2 = 16384 chains of 8192 spins (1.3e8 chain-updates per sweep, near
    the headline's 1.0e8)."""
    out = []
    for g in range(n_graphs):
        edges, _ = random_regular_edges(n, z, seed * 1000003 + g, bipartite=True)
        rng = np.random.default_rng(seed * 1000003 + g)
        for k in range(samples):
            J = np.where(rng.random(len(edges)) < 0.5, -1, 1).astype(np.int8)
            out.append(VbDesc(n=n, T=temps[k % len(temps)], seed=seed, instance_id=samples * g + k, graph_id=g,
                              n_replicas=2, edges=edges, J=J))
    return out


def vb_rrbg_batched(n_graphs: int = 256, n: int = 65536, z: int = 4, temps=(0.6, 0.8, 1.2),
                    seed: int = 6) -> List[VbDesc]:
    out = []
    for s in range(n_graphs):
        edges, J = random_regular_edges(n, z, seed * 1000003 + s, bipartite=True)
        for tau, T in enumerate(temps):
            out.append(VbDesc(n=n, T=T, seed=seed, instance_id=len(temps) * s + tau, graph_id=s,
                              n_replicas=2, edges=edges, J=J))
    return out
