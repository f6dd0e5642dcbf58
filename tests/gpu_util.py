"""Helpers for the GPU parity tests: run the oracle on a descriptor and
compare the library's observables with it element by element (all integer
quantities, so the bar is exact equality)."""
import numpy as np

import oracle
import paper_1906_11195_amd as sg


def require_gpu():
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    sg.library()          # raises if the HIP library is missing


def oracle_vb(d, n_sweeps, t_max):
    if d.edges is None:
        eu, ev, J = oracle.vb_instance(d.n, d.c, d.seed, d.graph_id)
    else:
        e = np.asarray(d.edges, np.int32).reshape(-1, 2)
        eu, ev, J = e[:, 0], e[:, 1], np.asarray(d.J, np.int8)
    return oracle.vb_run(d.n, eu, ev, J, d.T, d.seed, d.instance_id, d.n_replicas, n_sweeps, t_max,
                         start=d.start, s0=d.s0)


def oracle_sk(d, n_sweeps, t_max):
    J = d.J if d.J is not None else oracle.sk_couplings(d.n, d.seed, d.graph_id)
    return oracle.sk_run(d.n, J, d.T, d.seed, d.instance_id, d.n_replicas, n_sweeps, t_max,
                         start=d.start, s0=d.s0)


def assert_instance_equal(res, i, ref, spins=True, label=""):
    K = len(ref["times"])
    assert np.array_equal(res["times"][:K], ref["times"]), label
    assert res["k_done"] == ref["k_done"], label
    for key in ("bond", "gram", "accepted"):
        got = res[key][i]
        want = ref[key]
        assert np.array_equal(got, want), "%s %s mismatch:\n got %s\nwant %s" % (label, key, got, want)
    if ref["overlap"].size:
        assert np.array_equal(res["overlap"][i], ref["overlap"]), label + " overlap"
    if spins:
        assert np.array_equal(res["spins"][i], ref["spins"]), label + " spins"
