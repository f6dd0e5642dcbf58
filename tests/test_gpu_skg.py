"""GPU parity of the SK dynamics with real (Gaussian) couplings against the
oracle (orc_skg_run).  Spins, accepted counts, overlaps and Gram matrices are
integers and must be equal; the real bond sums B = sum_{i<j} J_ij s_i s_j are
summed in another order on each side and must agree within 1e-9 (the
rounding of ~N^2/2 double additions of terms below 1 is below 1e-12).  The
fields are double on both sides and each flip's change 2 s_i J_ij is exact, so
decisions can only differ if a 32-bit uniform equals the one integer that the
last-bit rounding of a threshold moves, an event of probability ~1e-14 per
decision."""
import concurrent.futures as cf
import math

import numpy as np
import pytest

import oracle
import paper_1906_11195_amd as sg
from paper_1906_11195_amd.workloads import gaussian_couplings
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

FLAGS = sg.MEASURE_OBS | sg.MEASURE_SPINS
BOND_TOL = 1e-9


def run_lib(descs, chunks, t_max):
    ctx = sg.sg_create_sk(descs, t_max=t_max)
    try:
        for k in chunks:
            sg.sg_sweep(ctx, k)
        return sg.sg_measure(ctx, FLAGS)
    finally:
        sg.sg_free(ctx)


def oracle_of(d, n_sweeps, t_max):
    return oracle.skg_run(d.n, d.Jf, d.T, d.seed, d.instance_id, d.n_replicas, n_sweeps, t_max,
                          period=d.recompute_period, start=d.start, s0=d.s0)


def check(descs, chunks, t_max):
    res = run_lib(descs, chunks, t_max)
    total = sum(chunks)
    with cf.ThreadPoolExecutor(max_workers=min(16, len(descs))) as ex:
        refs = list(ex.map(lambda d: oracle_of(d, total, t_max), descs))
    for i, ref in enumerate(refs):
        lab = "inst %d (n=%d, T=%s)" % (i, descs[i].n, descs[i].T)
        K = len(ref["times"])
        assert res["k_done"] == ref["k_done"], lab
        assert np.array_equal(res["spins"][i], ref["spins"]), lab + " spins"
        assert np.array_equal(res["accepted"][i], ref["accepted"]), lab + " accepted"
        assert np.array_equal(res["gram"][i], ref["gram"]), lab + " gram"
        if ref["overlap"].size:
            assert np.array_equal(res["overlap"][i], ref["overlap"]), lab + " overlap"
        assert np.all(res["bond"][i] == 0), lab + " integer bond unused"
        assert np.abs(res["bond_real"][i][:, :K] - ref["bond"]).max() < BOND_TOL, lab + " bond"
    return res, refs


@pytest.mark.parametrize("n", [2, 5, 63, 64, 65, 300, 1000])
def test_skg_ragged_sizes(n):
    require_gpu()
    J = gaussian_couplings(n, seed=n)
    descs = [sg.SkDesc(n=n, T=T, seed=3, instance_id=k, graph_id=0, Jf=J) for k, T in
             enumerate([0.5, 1.5, 0.0, math.inf])]
    check(descs, [40, 50, 40], 128)


def test_skg_starts_periods_and_separate_matrices():
    require_gpu()
    n = 257
    rng = np.random.default_rng(4)
    s0 = rng.choice([-1, 1], size=(2, n)).astype(np.int8)
    Ja, Jb = gaussian_couplings(n, seed=1), gaussian_couplings(n, seed=2)
    for period in (1, 16):
        descs = [sg.SkDesc(n=n, T=0.6, seed=5, instance_id=0, Jf=Ja, recompute_period=period),
                 sg.SkDesc(n=n, T=0.6, seed=5, instance_id=1, Jf=Jb, start=sg.START_ALIGNED,
                           recompute_period=period),
                 sg.SkDesc(n=n, T=0.9, seed=6, instance_id=2, Jf=Ja, start=sg.START_GIVEN, s0=s0,
                           recompute_period=period)]
        check(descs, [33, 1, 30], 64)


def test_skg_full_size_prefix():
    # the benchmark's shape (N = 4096, T = 0.5), a few samples over a prefix
    require_gpu()
    n = 4096
    descs = [sg.SkDesc(n=n, T=0.5, seed=7, instance_id=s, graph_id=s, Jf=gaussian_couplings(n, seed=90 + s))
             for s in range(3)]
    check(descs, [6], 8)


def test_skg_binary_values_equal_the_binary_path():
    # couplings +-1/sqrt(N) with 1/sqrt(N) = 2^-4 exact: the real path must
    # give the binary path's trajectory
    require_gpu()
    n = 256
    Jb = sg.sg_sk_inspect(sg.SkDesc(n=n, T=0.5, seed=3, instance_id=0, graph_id=6))[0]
    Jr = (Jb.astype(np.float32) / np.float32(16.0)).astype(np.float32)
    a = run_lib([sg.SkDesc(n=n, T=0.5, seed=3, instance_id=0, graph_id=6)], [100], 128)
    b = run_lib([sg.SkDesc(n=n, T=0.5, seed=3, instance_id=0, Jf=Jr)], [100], 128)
    assert np.array_equal(a["spins"][0], b["spins"][0])
    assert np.array_equal(a["accepted"], b["accepted"]) and np.array_equal(a["gram"], b["gram"])
    assert np.abs(b["bond_real"] - a["bond"] / 16.0).max() < BOND_TOL


def test_skg_corrupted_field_is_reported_by_the_recompute():
    require_gpu()
    n = 200
    d = sg.SkDesc(n=n, T=0.5, seed=3, instance_id=2, Jf=gaussian_couplings(n, seed=3), recompute_period=32)
    ctx = sg.sg_create_sk([d], t_max=128)
    try:
        sg.sg_sweep(ctx, 32)
        sg.sg_sk_corrupt_field(ctx, 0, 0, 17, 1)
        sg.sg_sweep(ctx, 31)
        assert sg.sg_measure(ctx, FLAGS, check=False)["status"] == sg.SG_OK
        sg.sg_sweep(ctx, 1)
        assert sg.sg_measure(ctx, FLAGS, check=False)["status"] == sg.SG_EPARITY
    finally:
        sg.sg_free(ctx)
    # mixing real and binary couplings in one context is refused
    with pytest.raises(sg.SgError):
        sg.sg_create_sk([d, sg.SkDesc(n=n, T=0.5, seed=3, instance_id=3)], t_max=8)


@pytest.mark.parametrize("n", [4100, 8192, 16384])
def test_skg_fields_beyond_one_pass(n):
    # a thread applies a block's flips to 4 fields at a time, so the 1024
    # threads of a chain cover 4096 fields per pass: 2 passes at N = 4100
    # and 8192, 4 at the largest size (whose fields fill most of the LDS)
    require_gpu()
    d = sg.SkDesc(n=n, T=0.5, seed=8, instance_id=0, graph_id=0, Jf=gaussian_couplings(n, seed=n + 1),
                  recompute_period=4)
    check([d], [3, 3], 8)
