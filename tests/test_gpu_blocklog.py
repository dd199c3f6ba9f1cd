"""GPU: the per-block log (temperature, residues, acceptance rate and sum-rule
drift after each block, the quantities the paper's program reports, Sec. 4).

Each record is the plain statistics of the walker population at its block
boundary: the test runs block by block, reads the residues and running
acceptance rates after every block and recomputes the statistics in numpy
(the definition); the records of the same anneal run in one call are
identical, and a ring smaller than the run keeps the newest records.
"""
import numpy as np
import pytest

from paper_1609_07936_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1609_07936_amd import sail
    sail.lib()
    return sail


def _setup(S, wl, prec, cap):
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(wl.n_walkers, wl.seed, precision=prec)
    gp.set_block_log(cap)
    return gp


@pytest.mark.parametrize("prec", [0, 1])
def test_block_log_is_the_population_statistics(S, prec):
    wl = W.small_64x32(n_sweeps=300, n_walkers=48 - prec)  # an even and an odd population (median)
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    every, branch = 10, 50
    gs = S.Schedule(T, branch_every=branch, resync_every=every)
    gp = _setup(S, wl, prec, 100)
    ref = []
    for k in range(0, wl.n_sweeps, every):
        gp.run(gs, k, every)
        chi2 = gp.read_chi2()
        rate = gp.read_state()["rate"]
        ref.append((chi2.min(), chi2.mean(), chi2.max(), rate.mean(), np.median(chi2)))
    ref = np.array(ref)
    log = gp.read_block_log()
    sweeps = np.arange(every, wl.n_sweeps + 1, every)
    assert log["total"] == sweeps.size
    np.testing.assert_array_equal(log["sweep"], sweeps)
    np.testing.assert_array_equal(log["event"], np.where(sweeps % branch == 0, sweeps // branch - 1, -1))
    np.testing.assert_array_equal(log["T"], T[sweeps - 1] * gp.chi2_unit)
    np.testing.assert_array_equal(log["chi2_min"], ref[:, 0])
    np.testing.assert_array_equal(log["chi2_max"], ref[:, 2])
    np.testing.assert_array_equal(log["chi2_median"], ref[:, 4])  # a selection: exact
    np.testing.assert_allclose(log["chi2_mean"], ref[:, 1], rtol=1e-14)
    np.testing.assert_allclose(log["rate_mean"], ref[:, 3], rtol=1e-14)
    # both sums are invariants of every move (Sec. 2.2): the drift a block
    # accumulates is rounding error
    assert np.all(log["drift_max"] >= 0) and np.all(log["drift_max"] < 1e-11), log["drift_max"]
    print(f"precision {prec}: {sweeps.size} records, largest drift {log['drift_max'].max():.2e}, "
          f"median residue {ref[0, 4]:.3e} -> {ref[-1, 4]:.3e}", flush=True)

    # the same anneal in one call gives the same records, and a ring of 4
    # keeps the newest 4 of them
    one = _setup(S, wl, prec, 100)
    one.run(gs, 0, wl.n_sweeps)
    ring = _setup(S, wl, prec, 4)
    ring.run(gs, 0, wl.n_sweeps)
    a, r = one.read_block_log(), ring.read_block_log()
    assert r["total"] == sweeps.size and r["sweep"].size == 4
    for f in ("sweep", "event", "T", "chi2_min", "chi2_mean", "chi2_median", "chi2_max", "rate_mean", "drift_max"):
        np.testing.assert_array_equal(a[f], log[f], err_msg=f)
        np.testing.assert_array_equal(r[f], log[f][-4:], err_msg=f)
    r2 = ring.read_block_log(max_records=2)
    np.testing.assert_array_equal(r2["sweep"], sweeps[-2:])


def test_block_log_switches(S):
    wl = W.small_64x32(n_sweeps=40, n_walkers=16)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    with pytest.raises(S.SailError) as e:
        gp.set_block_log(4)
    assert e.value.status == 6
    gp.init_walkers(wl.n_walkers, wl.seed)
    with pytest.raises(S.SailError) as e:
        gp.read_block_log()
    assert e.value.status == 6
    gp.set_block_log(4)
    gs = S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, 40), branch_every=20, resync_every=10)
    gp.run(gs, 0, 20)
    assert gp.read_block_log()["total"] == 2
    gp.set_block_log(4)  # a new call empties the log
    assert gp.read_block_log()["total"] == 0
    gp.set_block_log(0)
    gp.run(gs, 20, 20)  # off: nothing recorded, nothing read
    with pytest.raises(S.SailError):
        gp.read_block_log()


def test_block_log_full_population(S):
    """16384 walkers (the largest population): the record of each block
    equals the statistics of the residues read back, the median exactly."""
    wl = W.small_64x32(n_sweeps=20, n_walkers=16384)
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    gs = S.Schedule(T, branch_every=10, resync_every=10)
    gp = _setup(S, wl, 0, 8)
    for k in (0, 10):
        gp.run(gs, k, 10)
        chi2 = gp.read_chi2()
        rec = gp.read_block_log(max_records=1)
        assert rec["sweep"][0] == k + 10 and rec["event"][0] == k // 10
        assert rec["chi2_min"][0] == chi2.min() and rec["chi2_max"][0] == chi2.max()
        assert rec["chi2_median"][0] == np.median(chi2)
        np.testing.assert_allclose(rec["chi2_mean"][0], chi2.mean(), rtol=1e-14)


def test_block_log_in_a_batch_equals_alone(S):
    """Problems that keep a block log and run in a batch (with a problem
    that keeps none, and the paper's smoothing) record what they record
    alone, bit for bit."""
    import torch
    jobs = W.batch_jobs(3, base_seed=6100, n_sweeps=300)
    precs = [0, 1, 0]
    scheds = [S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), branch_every=wl.branch_every,
                         resync_every=wl.resync_every, smooth=0.01 * (i == 2)) for i, wl in enumerate(jobs)]

    def mk(i, log):
        wl = jobs[i]
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.init_walkers(wl.n_walkers, wl.seed, precision=precs[i])
        if log:
            gp.set_block_log(64)
        return gp

    alone = [mk(i, i != 1) for i in range(3)]
    for gp, sc, wl in zip(alone, scheds, jobs):
        gp.run(sc, 0, wl.n_sweeps)
    mixed = [mk(i, i != 1) for i in range(3)]
    S.Batch(mixed).run(scheds, 0, [wl.n_sweeps for wl in jobs])
    torch.cuda.synchronize()
    for i in (0, 2):
        a, b = alone[i].read_block_log(), mixed[i].read_block_log()
        assert a["total"] == b["total"] == jobs[i].n_sweeps // jobs[i].resync_every
        for f in ("sweep", "event", "T", "chi2_min", "chi2_mean", "chi2_median", "chi2_max", "rate_mean", "drift_max"):
            np.testing.assert_array_equal(b[f], a[f], err_msg=f"job {i} {f}")
    with pytest.raises(S.SailError):
        mixed[1].read_block_log()
