"""CPU tests of the C-ABI library: it loads, exports what include/sg.h
declares, and its host-side instance builder (graph, colouring, sweep order,
adjacency in sweep order, thresholds, SK couplings) equals the oracle's
independently built tables bit for bit.  No GPU is touched."""
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_1906_11195_amd as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "sg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(sg_\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if not n.endswith("_fn")))


def test_library_exports_every_declared_symbol():
    lib = sg.library()
    declared = _declared_functions()
    assert set(declared) >= {"sg_create_vb", "sg_create_sk", "sg_sweep", "sg_measure", "sg_free"}
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(sg.EXPORTS)


def test_strerror_and_null_handling():
    assert sg.sg_strerror(0) == "ok"
    assert "invalid" in sg.sg_strerror(sg.SG_EINVAL)
    lib = sg.library()
    lib.sg_free(None)                                      # no-op
    assert lib.sg_sweep(None, 1, None) == sg.SG_EINVAL
    assert lib.sg_measure(None, 1, None, None) == sg.SG_EINVAL
    assert lib.sg_create_vb(None, 1, None, None) == sg.SG_EINVAL


def _decode(tab, n):
    """Adjacency from the library's sweep-order tables, in vertex ids."""
    order = tab["order"]
    nbrs = {}
    for p in range(n):
        v = int(order[p])
        ents = tab["entries"][tab["row_start"][p]:tab["row_start"][p + 1]]
        nbrs[v] = sorted((int(order[e & 0x7FFFFFFF]), -1 if e >> 31 else 1) for e in ents)
    return nbrs


@pytest.mark.parametrize("n,c,seed,gid", [(1024, 4.0, 1, 0), (5000, 4.0, 2, 17), (777, 3.0, 9, 3)])
def test_vb_tables_equal_oracle(n, c, seed, gid):
    d = sg.VbDesc(n=n, T=0.8, seed=seed, instance_id=0, graph_id=gid, c=c)
    tab = sg.sg_vb_inspect(d)
    eu, ev, J, _ = oracle.er_graph(n, oracle.n_edges(n, c), seed, gid)
    assert np.array_equal(tab["edges"][:, 0], eu) and np.array_equal(tab["edges"][:, 1], ev)
    assert np.array_equal(tab["J"], J)
    colour, ncol = oracle.greedy_colour(n, eu, ev)
    assert np.array_equal(tab["colour"], colour) and tab["n_colours"] == ncol
    assert np.array_equal(tab["order"], oracle.sweep_order(colour, ncol, oracle.degrees(n, eu, ev)))
    nb = _decode(tab, n)
    ref = {v: [] for v in range(n)}
    for u, v, j in zip(eu.tolist(), ev.tolist(), J.tolist()):
        ref[u].append((v, j))
        ref[v].append((u, j))
    for v in range(n):
        assert nb[v] == sorted(ref[v])
    deg = np.bincount(np.concatenate([eu, ev]), minlength=n)
    assert tab["max_degree"] == deg.max()


@pytest.mark.parametrize("T", [0.5, 0.6, 0.8, 1.0, 1.2, 3.0, math.inf, 0.0])
def test_vb_thresholds_equal_oracle(T):
    d = sg.VbDesc(n=64, T=T, seed=1, instance_id=0)
    assert np.array_equal(sg.sg_vb_inspect(d)["thr"], oracle.thresholds(T, 1.0, 63))


@pytest.mark.parametrize("n,T", [(300, 0.5), (1000, 0.9), (4096, 0.5), (257, math.inf)])
def test_sk_tables_equal_oracle(n, T):
    d = sg.SkDesc(n=n, T=T, seed=3, instance_id=0, graph_id=5)
    J, thr = sg.sg_sk_inspect(d)
    if n <= 1000:
        assert np.array_equal(J, oracle.sk_couplings(n, 3, 5))
    else:
        rows = [0, 1, 63, 64, 2047, n - 1]
        full = oracle.sk_couplings(n, 3, 5)
        assert np.array_equal(J[rows], full[rows])
    assert np.array_equal(thr, oracle.thresholds(T, 1.0 / math.sqrt(n), n - 1))


def test_explicit_edges_copied_and_validated():
    n = 50
    eu, ev, J = oracle.vb_instance(n, 4.0, seed=4, graph_id=1)
    edges = np.stack([eu, ev], axis=1)
    d = sg.VbDesc(n=n, T=1.0, seed=1, instance_id=0, edges=edges, J=J)
    tab = sg.sg_vb_inspect(d)
    assert np.array_equal(tab["edges"], edges) and np.array_equal(tab["J"], J)
    bad = [edges.copy() for _ in range(3)]
    bad[0][0] = bad[0][1]                      # repeated pair
    bad[1][0, 1] = bad[1][0, 0]                # self-loop
    bad[2][0, 0] = n                           # out of range
    for b in bad:
        with pytest.raises(sg.SgError) as e:
            sg.sg_vb_inspect(sg.VbDesc(n=n, T=1.0, seed=1, instance_id=0, edges=b, J=J))
        assert e.value.code == sg.SG_EINVAL
    Jb = J.copy()
    Jb[3] = 2
    with pytest.raises(sg.SgError):
        sg.sg_vb_inspect(sg.VbDesc(n=n, T=1.0, seed=1, instance_id=0, edges=edges, J=Jb))


def test_descriptor_limits():
    with pytest.raises(sg.SgError) as e:
        sg.sg_vb_inspect(sg.VbDesc(n=(1 << 20) + 1, T=1.0, seed=1, instance_id=0))
    assert e.value.code == sg.SG_ENOTSUP
    for kw in (dict(n=1), dict(n=100, T=-1.0), dict(n=100, T=float("nan")), dict(n=100, n_replicas=9),
               dict(n=100, n_replicas=0), dict(n=100, start=7)):
        args = dict(n=100, T=1.0, seed=1, instance_id=0)
        args.update(kw)
        with pytest.raises(sg.SgError) as e:
            sg.sg_vb_inspect(sg.VbDesc(**args))
        assert e.value.code == sg.SG_EINVAL
    with pytest.raises(sg.SgError) as e:
        sg.sg_sk_inspect(sg.SkDesc(n=40000, T=1.0, seed=1, instance_id=0))
    assert e.value.code == sg.SG_ENOTSUP
    J = oracle.sk_couplings(16, 1, 1)
    J[0, 1] = -J[0, 1]                          # not symmetric
    with pytest.raises(sg.SgError):
        sg.sg_sk_inspect(sg.SkDesc(n=16, T=1.0, seed=1, instance_id=0, J=J))


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; covered by the GPU tests")
    with pytest.raises(sg.SgError) as e:
        sg.sg_create_vb([sg.VbDesc(n=64, T=1.0, seed=1, instance_id=0)], t_max=4, torch_alloc=False)
    assert e.value.code == sg.SG_EDEVICE


def test_resume_options_checked_before_the_device():
    # sg_opts.t_start: 0 <= t_start < 2^32, and no windowed correlation
    d = [sg.VbDesc(n=64, T=1.0, seed=1, instance_id=0)]
    for ts in (-1, 1 << 32):
        with pytest.raises(sg.SgError) as e:
            sg.sg_create_vb(d, t_max=4, torch_alloc=False, t_start=ts)
        assert e.value.code == sg.SG_EINVAL
    with pytest.raises(sg.SgError) as e:
        sg.sg_create_vb(d, t_max=4, torch_alloc=False, t_start=2, window_tw_max=1)
    assert e.value.code == sg.SG_ENOTSUP
