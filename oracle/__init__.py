"""Plain CPU oracle for the aging Metropolis dynamics (VB and SK spin glasses).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never links, imports or calls it; the two share no code.

The arithmetic lives in ``sg_oracle.c`` (plain sequential C, compiled with gcc
into ``oracle/_build/libsg_oracle.so``); this module only marshals numpy arrays
through ctypes.  Every function cites the passage it follows in the C source.

Passages of the paper (arXiv:1906.11195) that the oracle follows:
  * SK Hamiltonian, Eq. (1); binary couplings +-1/sqrt(N), SI section on the SK
    model; fixed update order and two clones, same section.
  * VB Hamiltonian, Eq. (3), couplings +-1.
  * Single-spin-flip Metropolis from a random start, time unit = one sweep:
    Methods; SI section on the bipartite random regular graph.
  * Parallel update by graph partition (bipartition generalised to a proper
    colouring): SI section "Simulations of the Bethe Lattice on GPUs".
  * Two-time correlation C(t,t') = (1/N) sum_i s_i(t) s_i(t'): introduction
    (definition of C and R) and SI Eq. formula1.

Parity status: every function is pinned by a ``-m "not gpu"`` test (see the
test files named ``test_oracle_*``); nothing here is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sg_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "libsg_oracle.so")
_lock = threading.Lock()
_lib = None

START_RANDOM, START_ALIGNED, START_GIVEN = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u32, u64, f64 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_philox4x64_10.argtypes = [P, P, P]
        lib.orc_accept_uniform.argtypes = [u64, u32, u32, u32, u64]
        lib.orc_accept_uniform.restype = u32
        lib.orc_init_spin.argtypes = [u64, u32, u32, u64]
        lib.orc_init_spin.restype = ctypes.c_int
        lib.orc_er_graph.argtypes = [i64, i64, u64, u32, P, P, P]
        lib.orc_er_graph.restype = i64
        lib.orc_sk_couplings.argtypes = [i64, u64, u32, P]
        lib.orc_greedy_colour.argtypes = [i64, i64, P, P, P]
        lib.orc_greedy_colour.restype = i32
        lib.orc_sweep_order.argtypes = [i64, P, i32, P, P]
        lib.orc_thresholds.argtypes = [f64, f64, i32, P]
        lib.orc_grid.argtypes = [i64, P]
        lib.orc_grid.restype = i32
        lib.orc_vb_run.argtypes = [i64, i64, P, P, P, f64, u64, u32, i32, i32, P, i64, i64, i32,
                                   P, P, P, P, P, P, P, i64, P, P]
        lib.orc_window_bin.argtypes = [u64]
        lib.orc_window_bin.restype = i32
        lib.orc_window_tw_count.argtypes = [i64, i64]
        lib.orc_window_tw_count.restype = i32
        lib.orc_vb_run.restype = ctypes.c_int
        lib.orc_sk_run.argtypes = [i64, P, f64, u64, u32, i32, i32, P, i64, i64, i32,
                                   P, P, P, P, P, P, P]
        lib.orc_sk_run.restype = ctypes.c_int
        lib.orc_skg_run.argtypes = [i64, P, f64, u64, u32, i32, i32, P, i64, i64, i32, i32,
                                    P, P, P, P, P, P, P, P]
        lib.orc_skg_run.restype = ctypes.c_int
        _lib = lib
        return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Philox and the stream layout
# --------------------------------------------------------------------------

def philox4x32(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox4x64(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def accept_uniform(seed, inst, rep, t, p) -> int:
    return int(_load().orc_accept_uniform(seed, inst, rep, t, p))


def init_spin(seed, inst, rep, p) -> int:
    return int(_load().orc_init_spin(seed, inst, rep, p))


# --------------------------------------------------------------------------
# Instances
# --------------------------------------------------------------------------

def n_edges(n: int, c: float) -> int:
    """M = floor(c N / 2) edges for mean degree c."""
    import math
    return int(math.floor(c * float(n) / 2.0))


def er_graph(n: int, m: int, seed: int, graph_id: int):
    """Erdos-Renyi G(N, M) with +-1 couplings; returns (eu, ev, J, attempts)."""
    eu = np.zeros(max(m, 1), dtype=np.int32)
    ev = np.zeros(max(m, 1), dtype=np.int32)
    J = np.zeros(max(m, 1), dtype=np.int8)
    a = _load().orc_er_graph(n, m, seed, graph_id, _ptr(eu), _ptr(ev), _ptr(J))
    if a < 0:
        raise ValueError("bad graph arguments")
    return eu[:m], ev[:m], J[:m], int(a)


def sk_couplings(n: int, seed: int, graph_id: int) -> np.ndarray:
    J = np.zeros((n, n), dtype=np.int8)
    _load().orc_sk_couplings(n, seed, graph_id, _ptr(J))
    return J


def greedy_colour(n: int, eu, ev):
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    colour = np.zeros(n, dtype=np.int32)
    ncol = _load().orc_greedy_colour(n, len(eu), _ptr(eu), _ptr(ev), _ptr(colour))
    return colour, int(ncol)


def sweep_order(colour, ncol: int, deg) -> np.ndarray:
    """Visiting order: colour classes in order, each by decreasing degree,
    ties by increasing vertex id."""
    colour = np.ascontiguousarray(colour, dtype=np.int32)
    deg = np.ascontiguousarray(deg, dtype=np.int32)
    order = np.zeros(len(colour), dtype=np.int32)
    _load().orc_sweep_order(len(colour), _ptr(colour), ncol, _ptr(deg), _ptr(order))
    return order


def degrees(n: int, eu, ev) -> np.ndarray:
    return np.bincount(np.concatenate([np.asarray(eu), np.asarray(ev)]), minlength=n).astype(np.int32)


def thresholds(T: float, de_scale: float, xmax: int) -> np.ndarray:
    thr = np.zeros(xmax + 1, dtype=np.uint64)
    _load().orc_thresholds(float(T), float(de_scale), int(xmax), _ptr(thr))
    return thr


def grid(t_max: int) -> np.ndarray:
    times = np.zeros(70, dtype=np.int64)
    k = _load().orc_grid(int(t_max), _ptr(times))
    return times[:k].copy()


# --------------------------------------------------------------------------
# Dynamics
# --------------------------------------------------------------------------

def _outputs(n, n_rep, K):
    npair = n_rep * (n_rep - 1) // 2
    return dict(times=np.zeros(K, np.int64), bond=np.zeros((n_rep, K), np.int64),
                overlap=np.zeros((max(npair, 1), K), np.int64),
                gram=np.zeros((n_rep, K, K), np.int64), accepted=np.zeros(n_rep, np.int64),
                spins=np.zeros((n_rep, n), np.int8), k=ctypes.c_int32(0))


def _finish(o, n_rep):
    k = o.pop("k").value
    npair = n_rep * (n_rep - 1) // 2
    o["overlap"] = o["overlap"][:npair]
    o["k_done"] = k
    return o


def window_bin(tau: int) -> int:
    """Minor-third interval of time tau >= 1 (see orc_window_bin)."""
    return int(_load().orc_window_bin(int(tau)))


def window_tw_count(t_max: int, tw_max: int) -> int:
    return int(_load().orc_window_tw_count(int(t_max), int(tw_max)))


def vb_run(n, eu, ev, J, T, seed, inst, n_rep, n_sweeps, t_max, start=START_RANDOM,
           s0=None, mode=0, window_tw_max=None):
    """One VB instance, n_rep replicas, n_sweeps sweeps (see orc_vb_run).  With
    window_tw_max, also the windowed correlation sums `window` [n_rep][kw][M]
    and their interval counts `window_count` [kw][M]."""
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    J = np.ascontiguousarray(J, dtype=np.int8)
    if s0 is not None:
        s0 = np.ascontiguousarray(s0, dtype=np.int8).reshape(n_rep, n)
    K = len(grid(t_max))
    o = _outputs(n, n_rep, K)
    win = cnt = None
    tw = -1
    if window_tw_max is not None:
        tw = int(window_tw_max)
        kw = window_tw_count(t_max, tw)
        nb = window_bin(t_max) + 1
        win = np.zeros((n_rep, kw, nb), np.int64)
        cnt = np.zeros((kw, nb), np.int64)
    rc = _load().orc_vb_run(n, len(eu), _ptr(eu), _ptr(ev), _ptr(J), float(T), seed, inst, n_rep,
                            start, _ptr(s0), n_sweeps, t_max, mode, _ptr(o["times"]),
                            _ptr(o["bond"]), _ptr(o["overlap"]), _ptr(o["gram"]),
                            _ptr(o["accepted"]), _ptr(o["spins"]), ctypes.byref(o["k"]),
                            tw, _ptr(win), _ptr(cnt))
    if rc != 0:
        raise ValueError("orc_vb_run rejected its arguments")
    out = _finish(o, n_rep)
    if win is not None:
        out["window"], out["window_count"] = win, cnt
    return out


def sk_run(n, J, T, seed, inst, n_rep, n_sweeps, t_max, start=START_RANDOM, s0=None,
           direct=False):
    """One SK instance (J int8 n x n), n_rep replicas (see orc_sk_run)."""
    J = np.ascontiguousarray(J, dtype=np.int8)
    if s0 is not None:
        s0 = np.ascontiguousarray(s0, dtype=np.int8).reshape(n_rep, n)
    K = len(grid(t_max))
    o = _outputs(n, n_rep, K)
    rc = _load().orc_sk_run(n, _ptr(J), float(T), seed, inst, n_rep, start, _ptr(s0), n_sweeps,
                            t_max, 1 if direct else 0, _ptr(o["times"]), _ptr(o["bond"]),
                            _ptr(o["overlap"]), _ptr(o["gram"]), _ptr(o["accepted"]),
                            _ptr(o["spins"]), ctypes.byref(o["k"]))
    if rc != 0:
        raise ValueError("orc_sk_run rejected its arguments")
    return _finish(o, n_rep)


def skg_run(n, J, T, seed, inst, n_rep, n_sweeps, t_max, period=64, start=START_RANDOM, s0=None,
            direct=False):
    """One SK instance with real couplings (J float32 n x n), n_rep replicas
    (see orc_skg_run): bond is the real sum B per replica and grid time,
    `fields` the final local fields."""
    J = np.ascontiguousarray(J, dtype=np.float32)
    if s0 is not None:
        s0 = np.ascontiguousarray(s0, dtype=np.int8).reshape(n_rep, n)
    K = len(grid(t_max))
    o = _outputs(n, n_rep, K)
    o["bond"] = np.zeros((n_rep, K), np.float64)
    h = np.zeros((n_rep, n), np.float64)
    rc = _load().orc_skg_run(n, _ptr(J), float(T), seed, inst, n_rep, start, _ptr(s0), n_sweeps,
                             t_max, int(period), 1 if direct else 0, _ptr(o["times"]), _ptr(o["bond"]),
                             _ptr(o["overlap"]), _ptr(o["gram"]), _ptr(o["accepted"]),
                             _ptr(o["spins"]), _ptr(h), ctypes.byref(o["k"]))
    if rc != 0:
        raise ValueError("orc_skg_run rejected its arguments")
    out = _finish(o, n_rep)
    out["fields"] = h
    return out


def vb_instance(n, c, seed, graph_id):
    """Generated VB instance: (eu, ev, J) for G(N, floor(cN/2)) from (seed, graph_id)."""
    eu, ev, J, _ = er_graph(n, n_edges(n, c), seed, graph_id)
    return eu, ev, J
