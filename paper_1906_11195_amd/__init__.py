"""Python binding of libsgmi.so, the gfx950 HIP library declared in include/sg.h.

Argument marshalling only: every step of the dynamics and of the measurements
runs in the library's HIP kernels.  PyTorch is used for device memory (its
caching allocator backs the library's allocation callbacks) and for streams.
There is no CPU fallback: if the library has not been built, every call raises.

The functions carry the C names (sg_create_vb, sg_create_sk, sg_sweep,
sg_measure, sg_free, sg_strerror, sg_vb_inspect, sg_sk_inspect).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import threading
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsgmi.so")

SG_OK, SG_EINVAL, SG_ENOMEM, SG_EDEVICE, SG_ESTATE, SG_EPARITY, SG_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
START_RANDOM, START_ALIGNED, START_GIVEN = 0, 1, 2
MEASURE_OBS, MEASURE_SPINS = 1, 2
OPT_AUTOTUNE, OPT_GRAPH, OPT_WINDOW, OPT_MULTISPIN, OPT_PLAIN_LDS = 1, 2, 4, 8, 16

EXPORTS = ("sg_create_vb", "sg_create_sk", "sg_sweep", "sg_measure", "sg_measure_noalloc", "sg_free",
           "sg_strerror", "sg_vb_inspect", "sg_sk_inspect", "sg_sk_corrupt_field")

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class _VbDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("c", ctypes.c_double), ("n_edges", ctypes.c_int64),
                ("edges", ctypes.c_void_p), ("J", ctypes.c_void_p), ("T", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("instance_id", ctypes.c_uint32),
                ("graph_id", ctypes.c_uint32), ("n_replicas", ctypes.c_int32),
                ("start", ctypes.c_int32), ("s0", ctypes.c_void_p)]


class _SkDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("J", ctypes.c_void_p), ("T", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("instance_id", ctypes.c_uint32),
                ("graph_id", ctypes.c_uint32), ("n_replicas", ctypes.c_int32),
                ("start", ctypes.c_int32), ("s0", ctypes.c_void_p),
                ("recompute_period", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("Jf", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("t_max", ctypes.c_int64), ("alloc", _ALLOC_FN), ("free", _FREE_FN),
                ("user", ctypes.c_void_p), ("chains_per_unit", ctypes.c_int32),
                ("threads_per_unit", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("split_members", ctypes.c_int32), ("window_tw_max", ctypes.c_int64),
                ("t_start", ctypes.c_int64)]


class _Obs(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n_replicas", ctypes.c_int32),
                ("k_cap", ctypes.c_int32), ("k_done", ctypes.c_int32), ("t_done", ctypes.c_int64),
                ("times", ctypes.c_void_p), ("bond", ctypes.c_void_p), ("overlap", ctypes.c_void_p),
                ("gram", ctypes.c_void_p), ("accepted", ctypes.c_void_p), ("spins", ctypes.c_void_p),
                ("kw", ctypes.c_int32), ("n_bins", ctypes.c_int32), ("window", ctypes.c_void_p),
                ("window_count", ctypes.c_void_p), ("bond_real", ctypes.c_void_p)]


class _VbTables(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int64), ("n_colours", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("edges", ctypes.c_void_p), ("J", ctypes.c_void_p),
                ("colour", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("row_start", ctypes.c_void_p), ("entries", ctypes.c_void_p),
                ("thr", ctypes.c_void_p)]


_lib = None
_lib_lock = threading.Lock()


def library() -> ctypes.CDLL:
    """Loads libsgmi.so; raises if it has not been built (no fallback)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsgmi.so is not built; run `python -m paper_1906_11195_amd.build` "
                               "(the HIP library is required, there is no CPU path)")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.sg_create_vb.argtypes = [P, ctypes.c_int32, P, P]
        lib.sg_create_vb.restype = ctypes.c_int32
        lib.sg_create_sk.argtypes = [P, ctypes.c_int32, P, P]
        lib.sg_create_sk.restype = ctypes.c_int32
        lib.sg_sweep.argtypes = [P, ctypes.c_int64, P]
        lib.sg_sweep.restype = ctypes.c_int32
        lib.sg_measure.argtypes = [P, ctypes.c_uint32, P, P]
        lib.sg_measure.restype = ctypes.c_int32
        lib.sg_measure_noalloc.argtypes = [P, P, P]
        lib.sg_measure_noalloc.restype = ctypes.c_int32
        lib.sg_free.argtypes = [P]
        lib.sg_free.restype = None
        lib.sg_strerror.argtypes = [ctypes.c_int32]
        lib.sg_strerror.restype = ctypes.c_char_p
        lib.sg_vb_inspect.argtypes = [P, P]
        lib.sg_vb_inspect.restype = ctypes.c_int32
        lib.sg_sk_inspect.argtypes = [P, P, P]
        lib.sg_sk_inspect.restype = ctypes.c_int32
        lib.sg_sk_corrupt_field.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
        lib.sg_sk_corrupt_field.restype = ctypes.c_int32
        _lib = lib
        return lib


class SgError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__("%s: %s (%d)" % (where, sg_strerror(code), code))
        self.code = code


def sg_strerror(code: int) -> str:
    return library().sg_strerror(int(code)).decode()


def _check(code: int, where: str):
    if code != SG_OK:
        raise SgError(code, where)


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# Descriptors
# --------------------------------------------------------------------------

@dataclasses.dataclass
class VbDesc:
    """One Viana-Bray instance (see sg_vb_desc in include/sg.h)."""
    n: int
    T: float
    seed: int
    instance_id: int
    graph_id: int = 0
    c: float = 4.0
    n_replicas: int = 2
    start: int = START_RANDOM
    edges: Optional[np.ndarray] = None     # [m, 2] int32
    J: Optional[np.ndarray] = None         # [m] int8
    s0: Optional[np.ndarray] = None        # [n_replicas, n] int8 (vertex order)


@dataclasses.dataclass
class SkDesc:
    """One Sherrington-Kirkpatrick instance (see sg_sk_desc in include/sg.h)."""
    n: int
    T: float
    seed: int
    instance_id: int
    graph_id: int = 0
    n_replicas: int = 2
    start: int = START_RANDOM
    J: Optional[np.ndarray] = None         # [n, n] int8 (binary couplings)
    s0: Optional[np.ndarray] = None
    recompute_period: int = 64
    Jf: Optional[np.ndarray] = None        # [n, n] float32 (real couplings)


def _vb_struct(d: VbDesc, keep: list) -> _VbDesc:
    s = _VbDesc()
    s.n, s.c, s.T = int(d.n), float(d.c), float(d.T)
    s.seed, s.instance_id, s.graph_id = int(d.seed), int(d.instance_id), int(d.graph_id)
    s.n_replicas, s.start = int(d.n_replicas), int(d.start)
    if d.edges is not None:
        e = np.ascontiguousarray(d.edges, dtype=np.int32).reshape(-1)
        j = np.ascontiguousarray(d.J, dtype=np.int8).reshape(-1)
        keep += [e, j]
        s.n_edges, s.edges, s.J = len(j), e.ctypes.data, j.ctypes.data
    if d.s0 is not None:
        s0 = np.ascontiguousarray(d.s0, dtype=np.int8).reshape(-1)
        keep.append(s0)
        s.s0 = s0.ctypes.data
    return s


def _sk_struct(d: SkDesc, keep: list) -> _SkDesc:
    s = _SkDesc()
    s.n, s.T = int(d.n), float(d.T)
    s.seed, s.instance_id, s.graph_id = int(d.seed), int(d.instance_id), int(d.graph_id)
    s.n_replicas, s.start, s.recompute_period = int(d.n_replicas), int(d.start), int(d.recompute_period)
    if d.J is not None:
        J = np.ascontiguousarray(d.J, dtype=np.int8).reshape(-1)
        keep.append(J)
        s.J = J.ctypes.data
    if d.Jf is not None:
        Jf = np.ascontiguousarray(d.Jf, dtype=np.float32).reshape(-1)
        keep.append(Jf)
        s.Jf = Jf.ctypes.data
    if d.s0 is not None:
        s0 = np.ascontiguousarray(d.s0, dtype=np.int8).reshape(-1)
        keep.append(s0)
        s.s0 = s0.ctypes.data
    return s


# --------------------------------------------------------------------------
# Device memory from torch's caching allocator
# --------------------------------------------------------------------------

def _torch_alloc(nbytes, user):
    import torch
    return int(torch.cuda.caching_allocator_alloc(int(nbytes)))


def _torch_free(ptr, nbytes, user):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


_ALLOC_CB = _ALLOC_FN(_torch_alloc)
_FREE_CB = _FREE_FN(_torch_free)


def _opts(t_max, chains_per_unit, threads_per_unit, torch_alloc, flags=0, split_members=0,
          window_tw_max=0, t_start=0):
    o = _Opts()
    o.t_max = int(t_max)
    o.t_start = int(t_start)
    o.window_tw_max = int(window_tw_max)
    o.chains_per_unit = int(chains_per_unit)
    o.threads_per_unit = int(threads_per_unit)
    o.flags = int(flags)
    o.split_members = int(split_members)
    if torch_alloc:
        o.alloc, o.free = _ALLOC_CB, _FREE_CB
    return o


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Context:
    """Owning handle of an sg_ctx."""

    def __init__(self, ptr, kind, ns, R, K, kw=0, n_bins=0, real=False):
        self.ptr = ptr
        self.kind = kind
        self.real = real        # SK with real couplings: bond_real instead of bond
        self.ns = list(ns)
        self.R = R
        self.K = K
        self.kw = kw            # windowed correlation: waiting times, intervals
        self.n_bins = n_bins

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                sg_free(self)
            except Exception:
                pass


def _grid_len(t_max):
    k = 1
    t = 1
    while t <= t_max:
        k += 1
        t <<= 1
    return k


def sg_create_vb(descs: Sequence[VbDesc], t_max: int, chains_per_unit: int = 0,
                 threads_per_unit: int = 0, torch_alloc: bool = True, autotune: bool = False,
                 graph: bool = False, split_members: int = 0,
                 window_tw_max: Optional[int] = None, multispin: bool = False,
                 plain_lds: bool = False, t_start: int = 0) -> Context:
    """window_tw_max: measure the windowed correlation with the grid times
    <= window_tw_max as waiting times (SG_OPT_WINDOW); multispin: pack the
    chains of a shared graph 64 per word (SG_OPT_MULTISPIN); plain_lds: keep
    no complemented copy of the spin words (SG_OPT_PLAIN_LDS); t_start:
    resume from start configurations at that time (sg_opts.t_start)."""
    keep = []
    arr = (_VbDesc * len(descs))(*[_vb_struct(d, keep) for d in descs])
    flags = (OPT_AUTOTUNE if autotune else 0) | (OPT_GRAPH if graph else 0)
    flags |= OPT_MULTISPIN if multispin else 0
    flags |= OPT_PLAIN_LDS if plain_lds else 0
    kw = n_bins = 0
    if window_tw_max is not None:
        flags |= OPT_WINDOW
        kw = _grid_len(min(int(window_tw_max), int(t_max)))   # grid times <= window_tw_max
        n_bins = (int(t_max) ** 4).bit_length()                # intervals of 1 .. t_max
    o = _opts(t_max, chains_per_unit, threads_per_unit, torch_alloc, flags, split_members,
              window_tw_max if window_tw_max is not None else 0, t_start)
    out = ctypes.c_void_p()
    _check(library().sg_create_vb(ctypes.byref(arr), len(descs), ctypes.byref(o), ctypes.byref(out)),
           "sg_create_vb")
    return Context(out, "vb", [d.n for d in descs], descs[0].n_replicas, _grid_len(t_max), kw, n_bins)


def sg_create_sk(descs: Sequence[SkDesc], t_max: int, threads_per_unit: int = 0,
                 torch_alloc: bool = True, t_start: int = 0) -> Context:
    """t_start: resume from start configurations at that time (sg_opts.t_start)."""
    keep = []
    arr = (_SkDesc * len(descs))(*[_sk_struct(d, keep) for d in descs])
    o = _opts(t_max, 0, threads_per_unit, torch_alloc, t_start=t_start)
    out = ctypes.c_void_p()
    _check(library().sg_create_sk(ctypes.byref(arr), len(descs), ctypes.byref(o), ctypes.byref(out)),
           "sg_create_sk")
    return Context(out, "sk", [d.n for d in descs], descs[0].n_replicas, _grid_len(t_max),
                   real=descs[0].Jf is not None)


def sg_sweep(ctx: Context, n_sweeps: int, stream=None) -> None:
    _check(library().sg_sweep(ctx.ptr, int(n_sweeps), _stream_handle(stream)), "sg_sweep")


def sg_measure(ctx: Context, flags: int = MEASURE_OBS, stream=None, check: bool = True) -> dict:
    """Observables as numpy arrays (shapes as documented for sg_obs)."""
    count, R, K = len(ctx.ns), ctx.R, ctx.K
    npair = R * (R - 1) // 2
    res = dict(times=np.zeros(K, np.int64), bond=np.zeros((count, R, K), np.int64),
               overlap=np.zeros((count, npair, K), np.int64),
               gram=np.zeros((count, R, K, K), np.int64), accepted=np.zeros((count, R), np.int64))
    o = _Obs()
    if flags & MEASURE_OBS:
        o.times, o.bond, o.gram = _p(res["times"]), _p(res["bond"]), _p(res["gram"])
        o.accepted = _p(res["accepted"])
        o.overlap = _p(res["overlap"]) if npair else None
    if ctx.real and flags & MEASURE_OBS:
        res["bond_real"] = np.zeros((count, R, K), np.float64)
        o.bond_real = _p(res["bond_real"])
    if ctx.kw and flags & MEASURE_OBS:
        res["window"] = np.zeros((count, R, ctx.kw, ctx.n_bins), np.int64)
        res["window_count"] = np.zeros((ctx.kw, ctx.n_bins), np.int64)
        o.window, o.window_count = _p(res["window"]), _p(res["window_count"])
    spins = None
    if flags & MEASURE_SPINS:
        spins = np.zeros(R * sum(ctx.ns), np.int8)
        o.spins = _p(spins)
    code = library().sg_measure(ctx.ptr, int(flags), ctypes.byref(o), _stream_handle(stream))
    res["status"] = code
    if code != SG_EPARITY or check:
        _check(code, "sg_measure")
    res["k_done"] = o.k_done
    res["t_done"] = o.t_done
    if spins is not None:
        out, base = [], 0
        for n in ctx.ns:
            out.append(spins[base:base + R * n].reshape(R, n))
            base += R * n
        res["spins"] = out
    return res


def sg_measure_noalloc(ctx: Context, stream=None, check: bool = True) -> dict:
    """The observables of sg_measure(ctx, MEASURE_OBS) through the entry point
    that allocates no memory (see include/sg.h); status in res["status"]."""
    count, R, K = len(ctx.ns), ctx.R, ctx.K
    npair = R * (R - 1) // 2
    res = dict(times=np.zeros(K, np.int64), bond=np.zeros((count, R, K), np.int64),
               overlap=np.zeros((count, npair, K), np.int64),
               gram=np.zeros((count, R, K, K), np.int64), accepted=np.zeros((count, R), np.int64))
    o = _Obs()
    o.times, o.bond, o.gram = _p(res["times"]), _p(res["bond"]), _p(res["gram"])
    o.accepted = _p(res["accepted"])
    o.overlap = _p(res["overlap"]) if npair else None
    if ctx.kw:
        res["window"] = np.zeros((count, R, ctx.kw, ctx.n_bins), np.int64)
        res["window_count"] = np.zeros((ctx.kw, ctx.n_bins), np.int64)
        o.window, o.window_count = _p(res["window"]), _p(res["window_count"])
    if ctx.real:
        res["bond_real"] = np.zeros((count, R, K), np.float64)
        o.bond_real = _p(res["bond_real"])
    code = library().sg_measure_noalloc(ctx.ptr, ctypes.byref(o), _stream_handle(stream))
    res["status"] = code
    if check:
        _check(code, "sg_measure_noalloc")
    res["k_done"] = o.k_done
    res["t_done"] = o.t_done
    return res


def sg_free(ctx: Context) -> None:
    if ctx.ptr:
        library().sg_free(ctx.ptr)
        ctx.ptr = None


def sg_vb_inspect(d: VbDesc) -> dict:
    keep = []
    s = _vb_struct(d, keep)
    t = _VbTables()
    _check(library().sg_vb_inspect(ctypes.byref(s), ctypes.byref(t)), "sg_vb_inspect")
    m, n = t.n_edges, d.n
    out = dict(edges=np.zeros((m, 2), np.int32), J=np.zeros(m, np.int8),
               colour=np.zeros(n, np.int32), order=np.zeros(n, np.int32),
               row_start=np.zeros(n + 1, np.int32), entries=np.zeros(2 * m, np.uint32),
               thr=np.zeros(64, np.uint64))
    for k in ("edges", "J", "colour", "order", "row_start", "entries", "thr"):
        setattr(t, k, out[k].ctypes.data)
    _check(library().sg_vb_inspect(ctypes.byref(s), ctypes.byref(t)), "sg_vb_inspect")
    out.update(n_colours=t.n_colours, max_degree=t.max_degree)
    return out


def sg_sk_inspect(d: SkDesc):
    keep = []
    s = _sk_struct(d, keep)
    J = np.zeros((d.n, d.n), np.int8)
    thr = np.zeros(d.n, np.uint64)
    _check(library().sg_sk_inspect(ctypes.byref(s), _p(J), _p(thr)), "sg_sk_inspect")
    return J, thr


def sg_sk_corrupt_field(ctx: Context, instance: int, replica: int, i: int, delta: int) -> None:
    """Fault injection for tests of the SK integrity check (see include/sg.h)."""
    _check(library().sg_sk_corrupt_field(ctx.ptr, int(instance), int(replica), int(i), int(delta)),
           "sg_sk_corrupt_field")
