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
from random_cases import random_case

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
    (4, 1, 16, 25, 200), (5, 1, 32, 0, 100), (6, 0, 16, 50, 125), (7, 1, 8, 150, 50),
    (8, 0, 4, 75, 125), (9, 1, 32, 0, 200),
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
    with pytest.raises(S.SailError):  # traced batch sweeps take uniform index selection
        batch.run(S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), walk_len=2), 0, 5)
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


def test_autotune_layout_alone_adds_the_smallest_tile(S):
    """For a problem with the device to itself the autotuner also times the
    smallest tile; its choice is cached apart from the shared one, so a
    shared call for the same shape still picks one of the two larger tiles."""
    import time
    wl = W.batch_jobs(1, base_seed=5151, n_sweeps=100)[0]
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    for prec, small, shared in ((S.SAIL_FP32, (8,), (16, 32)), (S.SAIL_FP64, (4,), (8, 16))):
        tpl = gp.autotune_layout(wl.n_walkers, prec, alone=True)
        assert tpl in small + shared
        gp.init_walkers(wl.n_walkers, wl.seed, precision=prec)
        assert gp.layout()[1] == tpl
        t0 = time.perf_counter()
        assert gp.autotune_layout(wl.n_walkers, prec, alone=True) == tpl
        assert time.perf_counter() - t0 < 0.05
        assert gp.autotune_layout(wl.n_walkers, prec) in shared


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


def _lockstep_bar(g_d, g_f, out, bar, tag):
    """Per-proposal residue changes within bar * M and identical accept bits
    (near-ties adopted by the oracle)."""
    err = np.abs(g_d - out["dchi2"])
    worst = float(np.max(err / np.maximum(out["cond"], 1e-300)))
    print(f"{tag}: worst |dchi2 error| / M over {err.size} proposals {worst:.3e}, "
          f"near-ties {out['near_ties']}", flush=True)
    assert out["hard_mismatch"] == 0, (tag, out["first_mismatch"])
    assert np.all(err <= bar * out["cond"]), (tag, worst)
    np.testing.assert_array_equal(g_f & 1, out["accept"] & 1, err_msg=tag)


def test_batched_jobs_against_the_oracle(S):
    """Jobs of the batched workload's distribution (fewer walkers, so that the
    oracle finishes in seconds) run in shared batch launches and are compared
    with the oracle directly, not through their solo runs:
      * two FP64 jobs (128 x 64 and 256 x 32, the second started alone and
        joining the batch at sweep 50) traced over all 300 sweeps: every
        proposal within 1e-12 M, identical accept bits, identical branching
        multipliers at the three events, final residues, spectra and the
        ensemble-mean spectrum at the anneal bars;
      * one FP32 job (128 x 128) whose state at sweep 100 (after its first
        event) is loaded into the oracle and replayed over the next resync
        segment, sweeps 100-149: every proposal within 1e-5 M of the FP64
        residue change;
      * two untraced jobs in the same launches end with the bits they have
        alone (the traced launch differs only by its trace stores)."""
    import torch
    import oracle as O
    pool = W.batch_jobs(64, base_seed=7000, n_sweeps=300)

    def pick(no, nt):
        return next(j for j in pool if j.omega.size == no and j.tau.size == nt)

    spec = [  # (workload, walkers, precision, tau per lane)
        (pick(128, 64), 64, S.SAIL_FP64, 16), (pick(256, 32), 48, S.SAIL_FP64, 8),
        (pick(128, 128), 128, S.SAIL_FP32, 16), (pick(512, 128), 256, S.SAIL_FP64, 16),
        (pick(1024, 256), 256, S.SAIL_FP32, 32)]
    scheds = [S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), branch_every=wl.branch_every,
                         resync_every=wl.resync_every) for wl, *_ in spec]

    def problem(wl, n, prec, tpl):
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.set_tau_per_lane(tpl)
        gp.init_walkers(n, wl.seed, precision=prec)
        gp.set_event_log(True)
        assert gp.layout()[1] == tpl
        return gp

    gps = [problem(*s) for s in spec]
    bufs = {}
    for i in (0, 1):
        wl, n = spec[i][0], spec[i][1]
        d = torch.zeros((n, 300, wl.omega.size), dtype=torch.float64, device="cuda")
        f = torch.zeros((n, 300, wl.omega.size), dtype=torch.uint8, device="cuda")
        gps[i].set_trace(0, 300, d.data_ptr(), f.data_ptr())
        bufs[i] = (d, f)
    gps[1].run(scheds[1], 0, 50)  # alone first, then in the batch
    batch = S.Batch(gps)
    batch.run(scheds, [0, 50, 0, 0, 0], [100, 50, 100, 100, 100])
    torch.cuda.synchronize()
    st32, chi32 = gps[2].read_state(), gps[2].read_chi2()
    wl32, n32 = spec[2][0], spec[2][1]
    d32 = torch.zeros((n32, 50, wl32.omega.size), dtype=torch.float64, device="cuda")
    f32 = torch.zeros((n32, 50, wl32.omega.size), dtype=torch.uint8, device="cuda")
    gps[2].set_trace(100, 150, d32.data_ptr(), f32.data_ptr())
    batch.run(scheds, [100, 100, 100, 100, 100], [200, 200, 50, 200, 100])
    torch.cuda.synchronize()

    # FP64 jobs: whole-anneal lockstep
    for i in (0, 1):
        wl, n = spec[i][0], spec[i][1]
        tag = f"batched FP64 job {wl.omega.size}x{wl.tau.size}"
        op = O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        an = O.Anneal(op, O.Schedule(scheds[i].T, branch_every=wl.branch_every, resync_every=wl.resync_every),
                      n, wl.seed)
        assert abs(gps[i].chi2_unit / an.chi2_unit - 1) < 1e-12
        g_d, g_f = (t.cpu().numpy() for t in bufs[i])
        ev = gps[i].read_events(3, multipliers=True)
        out = an.run(0, 300, trace=(0, 300), replay=g_f, replay_m=ev["m"])
        _lockstep_bar(g_d, g_f, out, 1e-12, tag)
        # identical multipliers but at logged near-ties (adopted by the oracle)
        assert out["branch_hard"] == 0, (tag, out["first_branch_mismatch"])
        np.testing.assert_array_equal(ev["m"], an.ev_m[:3], err_msg=tag)
        rob = an.ev_robust[:3] == 1
        np.testing.assert_array_equal(ev["status"][rob], an.ev_status[:3][rob], err_msg=tag)
        np.testing.assert_array_equal(ev["z"][rob], an.ev_z[:3][rob], err_msg=tag)
        print(f"{tag}: branching near-ties {out['branch_near_ties']}", flush=True)
        np.testing.assert_allclose(gps[i].read_chi2(), an.chi2, rtol=1e-9, err_msg=tag)
        st = gps[i].read_state()
        np.testing.assert_allclose(st["a"], an.a, rtol=1e-9, atol=1e-12 * np.abs(an.a).max(), err_msg=tag)
        np.testing.assert_allclose(st["F"], an.F, rtol=1e-12, err_msg=tag)
        dw = wl.omega[1] - wl.omega[0]
        assert np.sum(np.abs(gps[i].read_spectrum() - an.mean_spectrum())) * dw <= 1e-10 * wl.m0, tag

    # FP32 job: one resync segment replayed from its batched state at sweep 100
    op = O.Problem(wl32.omega, wl32.tau, wl32.Ft, wl32.sigma, wl32.m0, wl32.m1)
    an = O.Anneal(op, O.Schedule(scheds[2].T, branch_every=wl32.branch_every, resync_every=wl32.resync_every),
                  n32, wl32.seed)
    an.a[:] = st32["a"]
    an.F[:] = st32["F"]
    an.chi2[:] = chi32
    an.rate[:] = st32["rate"]
    an.args.chi2_unit = gps[2].chi2_unit
    g_d, g_f = d32.cpu().numpy(), f32.cpu().numpy()
    out = an.run(100, 150, trace=(100, 150), replay=g_f, band=1e-5)
    _lockstep_bar(g_d, g_f, out, 1e-5, "batched FP32 job 128x128, sweeps 100-149")
    st = gps[2].read_state()
    np.testing.assert_allclose(st["a"], an.a, rtol=1e-9, atol=1e-12 * np.abs(an.a).max())
    np.testing.assert_allclose(gps[2].read_chi2(), an.chi2, rtol=1e-9)

    # untraced jobs of the traced launches equal their solo runs
    for i, (k1, tag) in ((3, (300, "FP64 512x128")), (4, (200, "FP32 1024x256"))):
        alone = problem(*spec[i])
        alone.run(scheds[i], 0, k1)
        _assert_same(_snapshot(alone, k1 // 100), _snapshot(gps[i], k1 // 100), tag)


def test_random_problems_in_one_batch_equal_alone(S):
    """The sixteen seeded random problems and protocols (each checked against
    the oracle alone by the parity tests), every third one with the FP32
    loop, the tile requests cycling through every tile of the precision and
    the library's choice, run together in one batch: each ends with the
    bits it has alone."""
    import torch
    cases = [random_case(i) for i in range(16)]
    precs = [1 if i % 3 == 2 else 0 for i in range(16)]
    tiles = [((4, 8, 16, 0) if precs[i] == 0 else (8, 16, 32, 0))[i % 4] for i in range(16)]

    def mk(wl, mode, sigma, prec, tpl):
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma if sigma else None, wl.m0, wl.m1, mode)
        gp.set_tau_per_lane(tpl)
        gp.init_walkers(wl.n_walkers, wl.seed, precision=prec)
        gp.set_event_log(True)
        return gp

    scheds = [S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), **kw) for wl, kw, _, _ in cases]
    alone = [mk(wl, mode, sigma, p, t) for (wl, kw, mode, sigma), p, t in zip(cases, precs, tiles)]
    used = {(p, gp.layout()[1]) for p, gp in zip(precs, alone)}
    assert {(0, 4), (0, 8), (0, 16), (1, 8), (1, 16), (1, 32)} <= used, used
    for gp, sc, (wl, _, _, _) in zip(alone, scheds, cases):
        gp.run(sc, 0, wl.n_sweeps)
    mixed = [mk(wl, mode, sigma, p, t) for (wl, kw, mode, sigma), p, t in zip(cases, precs, tiles)]
    S.Batch(mixed).run(scheds, 0, [wl.n_sweeps for wl, _, _, _ in cases])
    torch.cuda.synchronize()
    for i, (gp_a, gp_b, (wl, kw, _, _)) in enumerate(zip(alone, mixed, cases)):
        n_ev = wl.n_sweeps // kw["branch_every"]
        _assert_same(_snapshot(gp_a, n_ev), _snapshot(gp_b, n_ev),
                     f"case {i} ({wl.omega.size}x{wl.tau.size}, {wl.n_walkers} walkers, prec {precs[i]})")


def test_autotune_cache_file_persists_across_processes(S, tmp_path):
    """With SAIL_TUNE_CACHE naming a file, a layout tuned in one process is
    appended to it as one line and a second process takes it from the file
    without timing anything (malformed lines are ignored); the choice for a
    problem with the device to itself is a line of its own tag."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    cache.write_text("not a tuning line\nsail-tune-v1 gfx950 1 2\n")
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "import torch; torch.cuda.init()\n"
            "from paper_1609_07936_amd import sail as S, workloads as W\n"
            "wl = W.batch_jobs(1, base_seed=4242, n_sweeps=100)[0]\n"
            "gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)\n"
            "t0 = time.perf_counter(); tpl = gp.autotune_layout(wl.n_walkers, S.SAIL_FP32)\n"
            "t1 = time.perf_counter(); tpa = gp.autotune_layout(wl.n_walkers, S.SAIL_FP32, alone=True)\n"
            "print(tpl, t1 - t0, tpa, time.perf_counter() - t1, flush=True)\n") % root
    env = dict(os.environ, SAIL_TUNE_CACHE=str(cache))
    runs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=180)
        assert r.returncode == 0, r.stderr[-2000:]
        tpl, dt, tpa, dta = r.stdout.split()
        runs.append((int(tpl), float(dt), int(tpa), float(dta)))
    text = cache.read_text().splitlines()
    for tag, col, cands in (("sail-tune-v1", 0, (16, 32)), ("sail-tune-alone-v1", 2, (8, 16, 32))):
        valid = [ln.split() for ln in text if ln.split()[:1] == [tag] and len(ln.split()) == 7]
        assert len(valid) == 1, (tag, valid)  # tuned once, appended once
        assert valid[0][1].startswith("gfx") and int(valid[0][6]) == runs[0][col] in cands
        assert runs[1][col] == runs[0][col] and runs[1][col + 1] < 0.05, runs


@pytest.mark.parametrize("n_walkers,prec,adaptive", [(256, 1, 0), (2048, 0, 1), (16384, 0, 0)])
def test_parallel_branch_search_matches_the_one_workgroup_search(S, n_walkers, prec, adaptive):
    """A single problem of 256 walkers or more searches Delta over many
    workgroups (Sec. 2.5, the fixed bracket-and-bisect search); a batch of one
    runs the one-workgroup search.  Ten events each: identical multipliers,
    Delta, P_r, zero counts, status, margins and walker state."""
    import torch
    wl = W.small_64x32(n_sweeps=100, n_walkers=n_walkers)
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    sc = S.Schedule(T, branch_every=10, resync_every=10, adaptive=adaptive)
    alone, one = (_problem(S, wl, prec, 16) for _ in range(2))
    alone.run(sc, 0, wl.n_sweeps)
    S.Batch([one]).run(sc, 0, wl.n_sweeps)
    torch.cuda.synchronize()
    a, b = _snapshot(alone, 10), _snapshot(one, 10)
    _assert_same(a, b, f"{n_walkers} walkers")
    for k in ("gap", "bracket"):
        np.testing.assert_array_equal(a[2][k], b[2][k], err_msg=k)
    assert np.all(a[2]["status"] == 0), a[2]["status"]
    print(f"{n_walkers} walkers: 10 events, zero counts {a[2]['z'].tolist()}", flush=True)


@pytest.mark.parametrize("eps0", [1e-7, 1e-300])
def test_parallel_branch_search_far_bracket(S, eps0):
    """A population whose residues span far more than the spread that sets
    Delta: 511 walkers a few tiny moves apart and one planted two-bin
    spectrum (both sum rules kept) with a residue ~20x theirs.  The crossing
    Delta lies beyond d0 2^16, so the parallel search needs its second
    bracketing round; event and state equal the one-workgroup search's bit
    for bit, and Delta and the multipliers equal the oracle's solve on the
    same residues and words (multipliers where the oracle finds the outcome
    robust, Sec. 2.5 near-ties).  With a vanishing move amplitude the 511
    residues stay equal, no Delta gives the target zero count, and both
    searches give up after the search's 200 doublings (status 1)."""
    import torch

    import oracle as O
    n = 512
    wl = W.small_64x32(n_sweeps=10, n_walkers=n)
    T = np.full(10, 1e-3)
    sc = S.Schedule(T, branch_every=3, resync_every=1, eps0=eps0)
    sc_nb = S.Schedule(T, branch_every=1000, resync_every=1, eps0=eps0)
    probs = [_problem(S, wl, 0, 16) for _ in range(3)]  # alone, batch of one, twin without branching
    blob = None
    for gp in probs:
        gp.run(sc, 0, 2)
        if blob is None:
            blob = bytearray(gp.state_export())
            a = gp.read_state()["a"]
            A, B = a[1].sum(), (wl.omega * a[1]).sum()
            p, s_ = 0, wl.omega.size - 1
            a_s = (B - wl.omega[p] * A) / (wl.omega[s_] - wl.omega[p])
            spike = np.zeros(wl.omega.size)
            spike[p], spike[s_] = A - a_s, a_s
            blob[48:48 + 8 * wl.omega.size] = spike.tobytes()  # walker 0's spectrum (scale 1 after the resync)
        gp.state_import(bytes(blob))
    alone, one, twin = probs
    alone.run(sc, 2, 1)
    S.Batch([one]).run(sc, 2, 1)
    twin.run(sc_nb, 2, 1)
    torch.cuda.synchronize()
    a_, b_ = _snapshot(alone, 1), _snapshot(one, 1)
    _assert_same(a_, b_, f"far bracket eps0 {eps0}")
    for k in ("gap", "bracket"):
        np.testing.assert_array_equal(a_[2][k], b_[2][k], err_msg=k)
    ev = a_[2]
    c = twin.read_chi2()
    d = ev["delta"][0]
    assert c.max() > 10 * c.min()
    if eps0 < 1e-100:
        assert np.ptp(np.sort(c)[:-1]) == 0.0
        assert ev["status"][0] == 1 and d == 0.0 and np.all(ev["m"][0] == 1)
        print(f"eps0 {eps0}: status 1 (target unreachable)", flush=True)
        return
    print(f"eps0 {eps0}: status {ev['status'][0]}, Delta (max - min) = 2^{np.log2(d * (c.max() - c.min())):.1f}",
          flush=True)
    assert ev["status"][0] == 0
    assert d * (c.max() - c.min()) > 2.0 ** 17  # beyond the first bracketing round
    res = O.branch_solve(c, O.branch_xi(wl.seed, 0, n), 0.25)
    assert res["status"] == 0 and not res["tie"]
    np.testing.assert_allclose(d, res["delta"], rtol=1e-9)
    if res["robust"]:
        np.testing.assert_array_equal(ev["m"][0], res["m"])
