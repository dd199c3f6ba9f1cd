"""GPU: the served-anneal loop.

A served job runs the batch rounds on its own device-resident state, so its
outputs (ensemble-mean spectrum, final residues, starting residue) are
bit-identical to the same job run alone through sail_run_schedule, which the
parity tests check against the oracle.  Admission keeps the footprint of the
in-flight jobs within the arena.
"""
import time

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


def _sched(S, wl):
    return S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), branch_every=wl.branch_every,
                      resync_every=wl.resync_every)


def _alone(S, wl, prec, tpl):
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    if tpl == S.AUTOTUNE:
        gp.autotune_layout(wl.n_walkers, prec)
    else:
        gp.set_tau_per_lane(tpl)
    gp.init_walkers(wl.n_walkers, wl.seed, precision=prec)
    gp.run(_sched(S, wl), 0, wl.n_sweeps)
    chi2 = gp.read_chi2()
    return {"mean": gp.read_spectrum(), "chi2_unit": gp.chi2_unit, "chi2_min": chi2.min(),
            "chi2_median": float(np.median(chi2))}


def test_served_jobs_match_alone(S):
    """Eight jobs of mixed sizes and precisions arrive in two waves while the
    first wave runs; every result equals the job run alone, bit for bit."""
    jobs = W.batch_jobs(8, base_seed=3000, n_sweeps=200)
    cfg = [(S.SAIL_FP32, S.AUTOTUNE), (S.SAIL_FP64, 16), (S.SAIL_FP32, 16), (S.SAIL_FP64, S.AUTOTUNE),
           (S.SAIL_FP32, 32), (S.SAIL_FP64, 8), (S.SAIL_FP32, S.AUTOTUNE), (S.SAIL_FP64, 16)]
    srv = S.Server(hbm_bytes=4 << 30, max_jobs=16)
    ids = []
    for i, (wl, (prec, tpl)) in enumerate(zip(jobs, cfg)):
        if i == 4:
            time.sleep(0.2)  # the second wave joins jobs already in flight
        ids.append(srv.submit(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1, wl.n_walkers, wl.seed, _sched(S, wl),
                              precision=prec, tau_per_lane=tpl))
    res = [srv.wait(j, timeout=120.0) for j in ids]
    st = srv.stats()
    srv.close()
    assert st["completed"] == 8 and st["failed"] == 0 and st["rounds"] > 0
    for r, wl, (prec, tpl) in zip(res, jobs, cfg):
        assert r["status"] == 0, r
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        ref = _alone(S, wl, prec, tpl)
        tag = f"{wl.name} {wl.omega.size}x{wl.tau.size} {wl.n_walkers} prec {prec} tpl {tpl}"
        np.testing.assert_array_equal(r["mean_spectrum"], ref["mean"], err_msg=tag)
        for k in ("chi2_unit", "chi2_min", "chi2_median"):
            assert r[k] == ref[k], (tag, k, r[k], ref[k])


def test_server_admission_within_budget(S):
    """An arena the size of the two largest jobs: six jobs all complete, the
    footprints in flight never exceed the arena, and a job larger than the
    arena is refused at submission."""
    jobs = W.batch_jobs(6, base_seed=4000, n_sweeps=100)
    scheds = [_sched(S, wl) for wl in jobs]
    foot = [S.Server.job_footprint(wl.omega, wl.tau, wl.n_walkers, sc, S.SAIL_FP32) for wl, sc in zip(jobs, scheds)]
    budget = sum(sorted(foot)[-2:])
    srv = S.Server(hbm_bytes=budget, max_jobs=8)
    big = next(j for j in W.batch_jobs(64, base_seed=4000, n_sweeps=100) if j.omega.size == 1024)
    assert S.Server.job_footprint(big.omega, big.tau, 16384, scheds[0], S.SAIL_FP32) > budget
    with pytest.raises(S.SailError):
        srv.submit(big.omega, big.tau, big.Ft, big.sigma, big.m0, big.m1, 16384, 1, scheds[0], precision=S.SAIL_FP32)
    ids = [srv.submit(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1, wl.n_walkers, wl.seed, sc,
                      precision=S.SAIL_FP32, tau_per_lane=16) for wl, sc in zip(jobs, scheds)]
    res = [srv.wait(j, timeout=120.0) for j in ids]
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in res)
    assert st["arena_peak"] <= st["arena_bytes"]
    # the footprints of the jobs in flight never exceed the arena
    events = sorted([(r["t_admit"], f) for r, f in zip(res, foot)] + [(r["t_done"], -f) for r, f in zip(res, foot)],
                    key=lambda e: (e[0], e[1]))
    held = np.cumsum([e[1] for e in events])
    assert held.max() <= st["arena_bytes"]
    assert held.max() < sum(foot)  # admission did hold jobs back


def test_server_timeout_and_shutdown(S):
    """A wait shorter than the job returns a timeout and leaves the job; the
    server shuts down with jobs queued and in flight."""
    wl = W.batch_jobs(1, base_seed=5000, n_sweeps=1000)[0]
    sc = _sched(S, wl)
    srv = S.Server(hbm_bytes=1 << 30, max_jobs=2)
    ids = [srv.submit(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1, wl.n_walkers, wl.seed + i, sc,
                      precision=S.SAIL_FP32, tau_per_lane=16) for i in range(6)]
    with pytest.raises(S.SailError) as e:
        srv.wait(ids[-1], timeout=0.01)
    assert e.value.status == S.SAIL_ETIMEOUT
    with pytest.raises(S.SailError):
        srv.wait(10 ** 9, timeout=0.01)
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 < 60


def test_served_protocol_matches_alone(S):
    """A served job with the paper's protocol (self-cooling, smoothing,
    adaptive branching, a two-step selection walk) beside a plain one: both
    equal their solo runs."""
    jobs = W.batch_jobs(2, base_seed=6000, n_sweeps=300)
    scheds = [S.Schedule(np.ones(300), branch_every=100, resync_every=50, smooth=0.01, adaptive=1, self_cool=1,
                         boil_blocks=1, cool_blocks=1, walk_len=2), _sched(S, jobs[1])]
    srv = S.Server(hbm_bytes=2 << 30, max_jobs=4)
    ids = [srv.submit(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1, wl.n_walkers, wl.seed, sc,
                      precision=S.SAIL_FP64, tau_per_lane=16) for wl, sc in zip(jobs, scheds)]
    res = [srv.wait(j, timeout=120.0) for j in ids]
    srv.close()
    for r, wl, sc in zip(res, jobs, scheds):
        assert r["status"] == 0, r
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.set_tau_per_lane(16)
        gp.init_walkers(wl.n_walkers, wl.seed, precision=S.SAIL_FP64)
        gp.run(sc, 0, 300)
        chi2 = gp.read_chi2()
        np.testing.assert_array_equal(r["mean_spectrum"], gp.read_spectrum())
        assert r["chi2_min"] == chi2.min() and r["chi2_median"] == float(np.median(chi2))


def test_served_job_against_the_oracle(S):
    """A served FP64 job (128 x 64, 64 walkers, 300 sweeps, three branching
    events), admitted while two larger FP32 jobs are in flight, compared
    directly with the oracle's run of the same job (which takes its own
    decisions: no replay): the starting residue within 1e-12, the final
    minimum and median residues within 1e-9 relative and the ensemble-mean
    spectrum within 1e-10 in L1, the anneal bars of the single-problem
    parity tests."""
    import oracle as O
    pool = W.batch_jobs(64, base_seed=8000, n_sweeps=300)
    small = next(j for j in pool if j.omega.size == 128 and j.tau.size == 64)
    big = [j for j in pool if j.omega.size >= 512][:2]
    sc = _sched(S, small)
    srv = S.Server(hbm_bytes=4 << 30, max_jobs=8)
    ids = [srv.submit(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1, 1024, wl.seed, _sched(S, wl),
                      precision=S.SAIL_FP32, tau_per_lane=16) for wl in big]
    time.sleep(0.1)
    mine = srv.submit(small.omega, small.tau, small.Ft, small.sigma, small.m0, small.m1, 64, small.seed, sc,
                      precision=S.SAIL_FP64, tau_per_lane=16)
    r = srv.wait(mine, timeout=120.0)
    others = [srv.wait(j, timeout=120.0) for j in ids]
    srv.close()
    assert r["status"] == 0 and all(o["status"] == 0 for o in others)
    op = O.Problem(small.omega, small.tau, small.Ft, small.sigma, small.m0, small.m1)
    an = O.Anneal(op, O.Schedule(sc.T, branch_every=small.branch_every, resync_every=small.resync_every), 64,
                  small.seed)
    out = an.run(0, 300)
    print(f"served FP64 job vs oracle: {out['proposals']} proposals, near-ties {out['near_ties']}", flush=True)
    assert abs(r["chi2_unit"] / an.chi2_unit - 1) < 1e-12
    assert abs(r["chi2_min"] / an.chi2.min() - 1) < 1e-9, (r["chi2_min"], an.chi2.min())
    assert abs(r["chi2_median"] / np.median(an.chi2) - 1) < 1e-9, (r["chi2_median"], np.median(an.chi2))
    dw = small.omega[1] - small.omega[0]
    assert np.sum(np.abs(r["mean_spectrum"] - an.mean_spectrum())) * dw <= 1e-10 * small.m0


def test_server_poll_and_cancel(S):
    """Per-job poll and cancel.  With two slots, four long jobs: the queued
    fourth is cancelled at once (its wait returns SAIL_ECANCELLED), the
    running first is cancelled in flight (it leaves at a round boundary, its
    arena block returns), and the other two complete with the bits they have
    alone.  Poll reports queued, running and done; cancelling a finished job
    is refused and an unknown id is rejected."""
    jobs = W.batch_jobs(4, base_seed=9000, n_sweeps=1000)
    sc = [_sched(S, wl) for wl in jobs]
    srv = S.Server(hbm_bytes=2 << 30, max_jobs=2)
    ids = [srv.submit(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1, 256, wl.seed, s, precision=S.SAIL_FP32,
                      tau_per_lane=16) for wl, s in zip(jobs, sc)]
    t0 = time.perf_counter()
    while srv.poll(ids[0]) != S.SAIL_JOB_RUNNING and time.perf_counter() - t0 < 30:
        time.sleep(0.001)
    assert srv.poll(ids[0]) == S.SAIL_JOB_RUNNING
    assert srv.poll(ids[3]) == S.SAIL_JOB_QUEUED
    srv.cancel(ids[3])
    assert srv.poll(ids[3]) == S.SAIL_JOB_DONE
    r3 = srv.wait(ids[3], timeout=1.0)
    assert r3["status"] == S.SAIL_ECANCELLED and r3["mean_spectrum"] is None
    srv.cancel(ids[0])
    r0 = srv.wait(ids[0], timeout=60.0)
    assert r0["status"] == S.SAIL_ECANCELLED
    res = [srv.wait(j, timeout=120.0) for j in ids[1:3]]
    with pytest.raises(S.SailError) as e:
        srv.wait(ids[0], timeout=0.0)  # already collected
    assert e.value.status == 1
    with pytest.raises(S.SailError) as e:
        srv.cancel(10 ** 9)
    assert e.value.status == 1
    # a job that has finished its anneal cannot be cancelled
    late = srv.submit(jobs[1].omega, jobs[1].tau, jobs[1].Ft, jobs[1].sigma, jobs[1].m0, jobs[1].m1, 64, 7,
                      _sched(S, jobs[1]), precision=S.SAIL_FP32, tau_per_lane=16)
    while srv.poll(late) != S.SAIL_JOB_DONE:
        time.sleep(0.005)
    with pytest.raises(S.SailError) as e:
        srv.cancel(late)
    assert e.value.status == S.SAIL_ESTATE
    assert srv.wait(late)["status"] == 0
    st = srv.stats()
    srv.close()
    assert st["cancelled"] == 2 and st["failed"] == 0 and st["completed"] == 3
    assert st["arena_used"] == 0
    for r, wl, s in zip(res, jobs[1:3], sc[1:3]):
        assert r["status"] == 0
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.set_tau_per_lane(16)
        gp.init_walkers(256, wl.seed, precision=S.SAIL_FP32)
        gp.run(s, 0, wl.n_sweeps)
        np.testing.assert_array_equal(r["mean_spectrum"], gp.read_spectrum())
