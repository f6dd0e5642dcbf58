"""Paper-level physics on the GPU (statistical, not parity): the VB model on
random regular graphs of degree 4 at T = 0.8 T_c, T_c = 1 / atanh(1 / sqrt 3),
quenched from random configurations, with 128 coupling samples x 2 replicas
per ensemble (multispin units of one graph and 32 samples).

  * The SI (bipartite-graph section) finds no statistically significant
    difference between bipartite and non-bipartite random regular graphs in
    C(t_w + t, t_w) at t_w = 4: the two ensembles' sample means agree within
    5 standard errors at every grid time.
  * Results and discussion: the correlation of a quench decays far below
    q_EA ~ 0.285 at large times (C(t_w + t, t_w) << q_EA), while it starts
    above it; the mean C(t_w + t, t_w) decreases with t.
"""
import math

import numpy as np
import pytest

import paper_1906_11195_amd as sg
from paper_1906_11195_amd.workloads import random_regular_edges
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

T_C = 1.0 / math.atanh(1.0 / math.sqrt(3.0))
Q_EA = 0.285


def ensemble(bipartite, n, graphs, samples, seed, t_max):
    descs = []
    for g in range(graphs):
        e, _ = random_regular_edges(n, 4, seed=seed * 1000 + g, bipartite=bipartite)
        rng = np.random.default_rng(seed * 1000 + g)
        for k in range(samples):
            J = np.where(rng.random(len(e)) < 0.5, -1, 1).astype(np.int8)
            descs.append(sg.VbDesc(n=n, T=0.8 * T_C, seed=seed, instance_id=g * samples + k, edges=e, J=J))
    ctx = sg.sg_create_vb(descs, t_max=t_max, multispin=True)
    try:
        sg.sg_sweep(ctx, t_max)
        res = sg.sg_measure(ctx, sg.MEASURE_OBS)
    finally:
        sg.sg_free(ctx)
    times = res["times"]
    kw = int(np.nonzero(times == 4)[0][0])
    # C(t_w + t, t_w) per chain for the grid times after t_w = 4
    ks = [k for k in range(len(times)) if times[k] > 4]
    C = res["gram"][:, :, kw, ks].reshape(-1, len(ks)) / float(n)
    return times[ks] - 4, C


def test_bipartite_and_random_regular_graphs_age_alike():
    require_gpu()
    n, t_max = 1 << 14, 1 << 14
    t, Cb = ensemble(True, n, 4, 32, seed=21, t_max=t_max)
    _, Cn = ensemble(False, n, 4, 32, seed=22, t_max=t_max)
    mb, mn = Cb.mean(0), Cn.mean(0)
    se = np.sqrt(Cb.var(0, ddof=1) / len(Cb) + Cn.var(0, ddof=1) / len(Cn))
    print("t", t.tolist(), "\nC bipartite", np.round(mb, 4).tolist(), "\nC random regular", np.round(mn, 4).tolist())
    assert np.all(np.abs(mb - mn) < 5 * se + 1e-12), (t, mb, mn, se)
    for C in (Cb, Cn):
        m = C.mean(0)
        s = np.sqrt(C.var(0, ddof=1) / len(C))
        # the correlation decays (no grid step rises by a significant amount)
        assert np.all(np.diff(m) < 3 * np.hypot(s[1:], s[:-1])), m
        assert m[0] > Q_EA and m[-1] < Q_EA, m    # from above q_EA to far below it
