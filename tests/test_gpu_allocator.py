"""GPU: device memory from the caller's allocator (sail_set_allocator).

With PyTorch's caching allocator behind the hook, the library's buffers
count in torch's memory statistics while they live and go back to it when
the objects are destroyed, also after the hook was changed in between.  The
allocator does not enter the arithmetic: every result equals the run on
hipMalloc'd memory bit for bit.
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
    yield sail
    sail.set_allocator(None, None)


def _sched(S, wl):
    return S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), branch_every=wl.branch_every,
                      resync_every=wl.resync_every)


def _problem(S, wl, prec):
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.set_tau_per_lane(16)
    gp.init_walkers(wl.n_walkers, wl.seed, precision=prec)
    return gp


def _results(gp):
    return gp.read_spectrum(), gp.read_chi2(), gp.chi2_unit


def _solve(S, jobs, precs):
    """One job alone, the rest as one batch; the results of each."""
    out = []
    gp = _problem(S, jobs[0], precs[0])
    gp.run(_sched(S, jobs[0]), 0, jobs[0].n_sweeps)
    out.append(_results(gp))
    gp.close()
    probs = [_problem(S, wl, p) for wl, p in zip(jobs[1:], precs[1:])]
    b = S.Batch(probs)
    b.run([_sched(S, wl) for wl in jobs[1:]], 0, [wl.n_sweeps for wl in jobs[1:]])
    out += [_results(pr) for pr in probs]
    b.close()
    for pr in probs:
        pr.close()
    return out


def test_torch_allocator_gives_identical_results(S):
    import torch
    torch.cuda.synchronize()
    jobs = W.batch_jobs(3, base_seed=5100, n_sweeps=200)
    precs = [S.SAIL_FP64, S.SAIL_FP32, S.SAIL_FP64]
    ref = _solve(S, jobs, precs)
    base = torch.cuda.memory_allocated()
    try:
        S.use_torch_allocator()
        got = _solve(S, jobs, precs)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
        # live buffers are counted by torch while the problem exists
        wl = jobs[0]
        gp = _problem(S, wl, S.SAIL_FP64)
        held = torch.cuda.memory_allocated() - base
        foot = S.footprint_bytes(wl.omega.size, wl.tau.size, wl.n_walkers, S.SAIL_FP64)
        assert held >= foot // 2, (held, foot)
        # a block made by the hook goes back to it after the hook is cleared
        S.use_torch_allocator(False)
        gp.run(_sched(S, wl), 0, wl.n_sweeps)
        again = _results(gp)
        gp.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        S.set_allocator(None, None)
    for (m0, c0, u0), (m1, c1, u1) in zip(ref, got):
        np.testing.assert_array_equal(m1, m0)
        np.testing.assert_array_equal(c1, c0)
        assert u1 == u0
    np.testing.assert_array_equal(again[0], ref[0][0])
    np.testing.assert_array_equal(again[1], ref[0][1])


def test_torch_allocator_backs_a_server_arena(S):
    import torch
    torch.cuda.synchronize()
    wl = W.batch_jobs(1, base_seed=5200, n_sweeps=100)[0]
    sc = _sched(S, wl)
    base = torch.cuda.memory_allocated()
    arena = 256 << 20
    try:
        S.use_torch_allocator()
        srv = S.Server(hbm_bytes=arena, max_jobs=4)
        assert torch.cuda.memory_allocated() - base >= arena
        j = srv.submit(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1, wl.n_walkers, wl.seed, sc,
                       precision=S.SAIL_FP32, tau_per_lane=16)
        r = srv.wait(j, timeout=120.0)
        srv.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        S.set_allocator(None, None)
    assert r["status"] == 0, r
    gp = _problem(S, wl, S.SAIL_FP32)
    gp.run(sc, 0, wl.n_sweeps)
    np.testing.assert_array_equal(r["mean_spectrum"], gp.read_spectrum())
    assert r["chi2_min"] == gp.read_chi2().min()
    gp.close()


def test_failing_allocator_reports_out_of_memory(S):
    """An allocator that returns nothing makes problem creation fail with
    SAIL_ENOMEM and leaves nothing behind."""
    wl = W.batch_jobs(1, base_seed=5300, n_sweeps=10)[0]
    try:
        S.set_allocator(lambda n, d: 0, lambda p, n, d: None)
        with pytest.raises(S.SailError) as e:
            gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
            gp.init_walkers(wl.n_walkers, wl.seed)
        assert e.value.status == 3
    finally:
        S.set_allocator(None, None)


def test_allocator_failing_midway_leaks_nothing(S):
    """An allocator that runs dry after k blocks, for k across the blocks
    walker initialisation takes: init fails with SAIL_ENOMEM, the problem
    stays usable (a later init with hipMalloc runs), and once it is
    destroyed every block the hook handed out has come back to it (torch's
    count returns to where it was)."""
    import torch
    wl = W.batch_jobs(1, base_seed=5400, n_sweeps=20)[0]
    live = {}

    def alloc_upto(k):
        calls = [0]

        def alloc(n, d):
            calls[0] += 1
            if calls[0] > k:
                return 0
            p = torch.cuda.caching_allocator_alloc(n, device=d)
            live[p] = n
            return p
        return alloc, calls

    def release(p, n, d):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    try:
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        alloc, calls = alloc_upto(10 ** 9)
        S.set_allocator(alloc, release)
        gp.init_walkers(wl.n_walkers, wl.seed)
        total = calls[0]
        assert total > 5 and len(live) == total
        gp.close()
        assert not live
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        for k in sorted({0, 1, total // 2, total - 1}):
            S.set_allocator(None, None)
            gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
            alloc, calls = alloc_upto(k)
            S.set_allocator(alloc, release)
            with pytest.raises(S.SailError) as e:
                gp.init_walkers(wl.n_walkers, wl.seed)
            assert e.value.status == 3, (k, e.value)
            S.set_allocator(None, None)
            with pytest.raises(S.SailError) as e:  # a failed initialisation leaves no walkers
                gp.run(S.Schedule(np.ones(10)), 0, 2)
            assert e.value.status == 6, (k, e.value)
            gp.init_walkers(wl.n_walkers, wl.seed)  # usable after the failure
            gp.run(S.Schedule(np.ones(10)), 0, 2)
            gp.close()
            assert not live, (k, len(live))  # whatever the hook handed out came back to it
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == base, k
    finally:
        S.set_allocator(None, None)


def test_failed_block_log_resize_keeps_the_old_log(S):
    """Switching the block log to a new capacity allocates the new ring
    before it drops the old one: when the allocation fails (SAIL_ENOMEM) the
    old log and its records stay as they were, and the next block appends."""
    wl = W.small_64x32(n_sweeps=40, n_walkers=16)
    gs = S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, 40), branch_every=20, resync_every=10)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(wl.n_walkers, wl.seed)
    gp.set_block_log(8)
    gp.run(gs, 0, 20)
    before = gp.read_block_log()
    assert before["total"] == 2
    try:
        S.set_allocator(lambda n, d: 0, lambda p, n, d: None)
        with pytest.raises(S.SailError) as e:
            gp.set_block_log(64)
        assert e.value.status == 3
    finally:
        S.set_allocator(None, None)
    after = gp.read_block_log()
    assert after["total"] == 2
    for f in ("sweep", "T", "chi2_min", "chi2_median"):
        np.testing.assert_array_equal(after[f], before[f])
    gp.run(gs, 20, 10)
    assert gp.read_block_log()["total"] == 3
    gp.close()


def test_failed_event_log_switch_keeps_the_old_multipliers(S):
    """Starting a new multiplier log allocates it before dropping the old
    one: when the allocation fails the multipliers of the events run so far
    stay readable, and events keep being logged."""
    wl = W.small_64x32(n_sweeps=60, n_walkers=16)
    gs = S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, 60), branch_every=20, resync_every=10)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(wl.n_walkers, wl.seed)
    gp.set_event_log(True)
    gp.run(gs, 0, 40)
    before = gp.read_events(2, multipliers=True)
    assert np.all(before["m"].sum(axis=1) == wl.n_walkers)
    try:
        S.set_allocator(lambda n, d: 0, lambda p, n, d: None)
        with pytest.raises(S.SailError) as e:
            gp.set_event_log(True)
        assert e.value.status == 3
    finally:
        S.set_allocator(None, None)
    np.testing.assert_array_equal(gp.read_events(2, multipliers=True)["m"], before["m"])
    gp.run(gs, 40, 20)
    ev = gp.read_events(3, multipliers=True)
    np.testing.assert_array_equal(ev["m"][:2], before["m"])
    assert ev["m"][2].sum() == wl.n_walkers
    gp.close()
