"""GPU: many problems annealed together in shared launches.

Every job of a batch runs the per-problem kernels on its own state with the
counter-based random stream of its own seed, so the bar is bit-identity with
the same job run alone through sail_run_schedule (which the parity tests
check against the oracle): spectra, reconstructions, acceptance rates,
residues and branching logs are compared with array_equal.
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


# (label, precision, tau points per lane, first sweep, sweeps)
MIX = [
    (0, 1, 16, 0, 200), (1, 1, 32, 50, 150), (2, 0, 16, 100, 100), (3, 0, 8, 0, 175),
    (4, 1, 16, 25, 200), (5, 1, 32, 0, 100), (6, 0, 16, 50, 125), (7, 1, 16, 150, 50),
    (8, 0, 8, 75, 125), (9, 1, 32, 0, 200),
]


def _jobs():
    """Ten jobs of the batched workload's distribution that cover all of its
    bin counts and time counts."""
    pool = W.batch_jobs(64, n_sweeps=400)
    pick, seen_o, seen_t = [], set(), set()
    for j in pool:
        if j.omega.size not in seen_o or j.tau.size not in seen_t:
            pick.append(j)
            seen_o.add(j.omega.size)
            seen_t.add(j.tau.size)
    pick += [j for j in pool if all(j is not q for q in pick)][:len(MIX) - len(pick)]
    assert len(pick) == len(MIX) and seen_o == {128, 256, 512, 1024} and seen_t == {32, 64, 128, 256}
    return pick


def _problem(S, wl, prec, tpl):
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.set_tau_per_lane(tpl)
    gp.init_walkers(wl.n_walkers, wl.seed, precision=prec)
    gp.set_event_log(True)
    assert gp.layout()[1] == tpl
    return gp


def _snapshot(gp, n_events):
    st = gp.read_state()
    ev = gp.read_events(n_events, multipliers=True)
    return st, gp.read_chi2(), ev


def _assert_same(a, b, tag):
    (sa, ca, ea), (sb, cb, eb) = a, b
    for k in ("a", "F", "rate"):
        np.testing.assert_array_equal(sa[k], sb[k], err_msg=f"{tag}: {k}")
    np.testing.assert_array_equal(ca, cb, err_msg=f"{tag}: chi2")
    for k in ("delta", "pr", "z", "status", "m"):
        np.testing.assert_array_equal(ea[k], eb[k], err_msg=f"{tag}: events {k}")


def test_batch_bit_identical_to_alone(S):
    """Ten jobs of mixed sizes, precisions and lane layouts, started at
    different sweeps of their schedules, run in one batch: each ends with the
    bits it has when run alone."""
    import torch
    jobs = _jobs()
    scheds = [S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), branch_every=wl.branch_every,
                         resync_every=wl.resync_every) for wl in jobs]
    alone, mixed = [], []
    for (ji, prec, tpl, k0, n), wl, sc in zip(MIX, jobs, scheds):
        for dst in (alone, mixed):
            gp = _problem(S, wl, prec, tpl)
            if k0:
                gp.run(sc, 0, k0)
            dst.append(gp)
    for gp, sc, (ji, prec, tpl, k0, n) in zip(alone, scheds, MIX):
        gp.run(sc, k0, n)
    batch = S.Batch(mixed)
    batch.set_timing(True)
    batch.run(scheds, [m[3] for m in MIX], [m[4] for m in MIX])
    torch.cuda.synchronize()
    ms, launches = batch.sweep_timing()
    assert launches > 0 and ms > 0
    for gp_a, gp_b, (ji, prec, tpl, k0, n), wl in zip(alone, mixed, MIX, jobs):
        n_ev = (k0 + n) // wl.branch_every
        _assert_same(_snapshot(gp_a, n_ev), _snapshot(gp_b, n_ev), f"job {ji} ({wl.omega.size}x{wl.tau.size}, "
                                                                    f"{wl.n_walkers} walkers, prec {prec}, tpl {tpl})")
        assert np.all(gp_b.read_events(n_ev)["status"] >= 0)


def test_batch_in_stages(S):
    """A batch run split over two calls equals the single-problem runs in one
    call (the round boundaries carry no state of their own)."""
    import torch
    jobs = _jobs()[:4]
    cfg = MIX[:4]
    scheds = [S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), branch_every=wl.branch_every,
                         resync_every=wl.resync_every) for wl in jobs]
    alone = [_problem(S, wl, m[1], m[2]) for wl, m in zip(jobs, cfg)]
    mixed = [_problem(S, wl, m[1], m[2]) for wl, m in zip(jobs, cfg)]
    for gp, sc in zip(alone, scheds):
        gp.run(sc, 0, 230)
    batch = S.Batch(mixed)
    batch.run(scheds, 0, 130)
    batch.run(scheds, 130, 100)
    torch.cuda.synchronize()
    for gp_a, gp_b, wl in zip(alone, mixed, jobs):
        _assert_same(_snapshot(gp_a, 2), _snapshot(gp_b, 2), wl.name)


def test_batch_errors(S):
    wl = W.small_64x32()
    sc = S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps))
    a = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    b = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    with pytest.raises(S.SailError):
        S.Batch([a, a])
    batch = S.Batch([a, b])
    a.init_walkers(16, 1)
    with pytest.raises(S.SailError) as e:  # b has no walkers
        batch.run(sc, 0, 10)
    assert e.value.status == 6
    b.init_walkers(16, 2)
    with pytest.raises(S.SailError):
        batch.run(sc, 0, wl.n_sweeps + 1)
    import torch
    d = torch.zeros((16, 2, wl.omega.size), dtype=torch.float64, device="cuda")
    f = torch.zeros((16, 2, wl.omega.size), dtype=torch.uint8, device="cuda")
    a.set_trace(0, 2, d.data_ptr(), f.data_ptr())
    with pytest.raises(S.SailError):
        batch.run(sc, 0, 5)
    a.set_trace(0, 0)
    with pytest.raises(S.SailError):  # a self-cooling run cannot start inside a block it never started
        batch.run(S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), self_cool=1), 50, 5)
    batch.run(sc, 0, 5)
    torch.cuda.synchronize()


def test_autotune_layout(S):
    """The autotuner picks one of the two candidate tiles, the next init uses
    it, and a second call for the same shape is served from the cache."""
    import time
    wl = W.batch_jobs(1, n_sweeps=100)[0]
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    for prec, cands in ((S.SAIL_FP32, (16, 32)), (S.SAIL_FP64, (8, 16))):
        tpl = gp.autotune_layout(wl.n_walkers, prec)
        assert tpl in cands
        gp.init_walkers(wl.n_walkers, wl.seed, precision=prec)
        assert gp.layout()[1] == tpl
        t0 = time.perf_counter()
        assert gp.autotune_layout(wl.n_walkers, prec) == tpl
        assert time.perf_counter() - t0 < 0.05


def test_batch_protocol_bit_identical_to_alone(S):
    """The paper's protocol in a batch: self-cooling, smoothing and adaptive
    branching on four jobs of mixed precisions and layouts, two of them with
    the Sec. 2.3 selection walk, run in two batch calls split inside a block,
    end with the bits of the same jobs run alone in one call."""
    import torch
    jobs = _jobs()[:4]
    cfg = MIX[:4]
    scheds = [S.Schedule(np.ones(400), branch_every=wl.branch_every, resync_every=wl.resync_every, smooth=0.01,
                         adaptive=1, self_cool=1, boil_blocks=1, cool_blocks=2, walk_len=2 * (i % 2))
              for i, wl in enumerate(jobs)]
    alone = [_problem(S, wl, m[1], m[2]) for wl, m in zip(jobs, cfg)]
    mixed = [_problem(S, wl, m[1], m[2]) for wl, m in zip(jobs, cfg)]
    for gp, sc in zip(alone, scheds):
        gp.run(sc, 0, 400)
    batch = S.Batch(mixed)
    batch.run(scheds, 0, 130)
    batch.run(scheds, 130, 270)
    torch.cuda.synchronize()
    for gp_a, gp_b, wl in zip(alone, mixed, jobs):
        _assert_same(_snapshot(gp_a, 4), _snapshot(gp_b, 4), wl.name)


def test_many_jobs_reach_a_branching_boundary_together(S):
    """256 small jobs reach a branching event in the same round with
    smoothing and adaptive branching on, so that round stages three resync
    descriptors and one branching descriptor per job (the largest round the
    staging slot must hold); every job ends with the bits it has alone
    (checked on a spread of them, in both precisions)."""
    import torch
    tgt = W.Target([1.2, 3.0], [0.3, 0.6], [0.5, 0.5], 6.0)
    tau = W.uniform_tau(0.05, 1.5, 8)
    base = W.make("many", 6.0, 16, tau, tgt, 1e-4, 21, 8, 200, 1e2, 1e-3, 100, 50, 0, n_quad=2000)
    T = W.geometric_schedule(base.t_hi, base.t_lo, base.n_sweeps)
    sc = S.Schedule(T, branch_every=100, resync_every=50, smooth=0.01, adaptive=1)
    n_jobs = 256

    def job(i):
        gp = S.Problem(base.omega, base.tau, base.Ft, base.sigma, base.m0, base.m1)
        gp.init_walkers(8, 5000 + i, precision=i % 2)
        gp.set_event_log(True)
        return gp

    mixed = [job(i) for i in range(n_jobs)]
    batch = S.Batch(mixed)
    batch.run(sc, 0, base.n_sweeps)
    torch.cuda.synchronize()
    for i in (0, 1, 2, 63, 128, 201, 254, 255):
        alone = job(i)
        alone.run(sc, 0, base.n_sweeps)
        _assert_same(_snapshot(alone, 2), _snapshot(mixed[i], 2), f"job {i}")
        assert np.all(mixed[i].read_events(2)["status"] == 0)
