"""GPU parity: the HIP library against the CPU oracle on the same seeded
inputs and the same Philox stream.

The bar (from the rounding of the residue change in both arithmetics):
  * |dchi2_gpu - dchi2_oracle| <= 1e-12 * M for every traced proposal, M the
    condition scale sum_i w_i (|r-1||F_i| + |dp|K_pi + |ds|K_si)(2|F_i| + 2|Ft_i| + |dF_i|);
  * identical accept decisions, except near-ties (decisions whose margin lies
    inside the 1e-12 band), which the oracle logs and adopts;
  * identical branching multipliers, targets and donors, except at a
    branching near-tie (an event whose oracle outcome changes when the
    residues are perturbed by 1e-9 relative), where the oracle logs and
    adopts the GPU's multipliers;
  * final residues within 1e-9 relative and the averaged spectrum within
    1e-10 in L1 (sum_j |da_j| d_omega, against a unit zeroth moment).
"""
import numpy as np
import pytest

import oracle as O
from paper_1609_07936_amd import workloads as W
from random_cases import random_case as _random_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1609_07936_amd import sail
    sail.lib()
    return sail


def _pair(S, wl, n_walkers, seed, sched_kw=None, mode=0, sigma=True, T=None, tpl=0):
    sched_kw = sched_kw or {}
    if T is None:
        T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    sg = wl.sigma if sigma else None
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, sg, wl.m0, wl.m1, mode)
    gp.set_tau_per_lane(tpl)
    gp.init_walkers(n_walkers, seed)
    op = O.Problem(wl.omega, wl.tau, wl.Ft, sg, wl.m0, wl.m1, mode)
    return gp, S.Schedule(T, **sched_kw), op, O.Schedule(T, **sched_kw)


def _trace_buffers(n, n_sweeps, n_omega):
    import torch
    d = torch.zeros((n, n_sweeps, n_omega), dtype=torch.float64, device="cuda")
    f = torch.zeros((n, n_sweeps, n_omega), dtype=torch.uint8, device="cuda")
    return d, f


def _check_trace(g_d, g_f, out):
    cond = out["cond"]
    err = np.abs(g_d - out["dchi2"])
    bad = err > 1e-12 * cond
    worst = float(np.max(err / np.maximum(cond, 1e-300)))
    print(f"worst |dchi2 error| / M over {err.size} proposals: {worst:.3e}", flush=True)
    assert not bad.any(), f"{bad.sum()} proposals outside 1e-12 M; worst {worst:.3e}"
    assert out["hard_mismatch"] == 0, f"hard mismatches at {out['first_mismatch']}"
    # after adopting near-ties the accept bits agree everywhere
    np.testing.assert_array_equal(g_f & 1, out["accept"] & 1)


def _check_branching(ev, an, out, n_ev, tag=""):
    """Identical multipliers at every event but logged near-ties (adopted by
    the oracle, which then reports them); status, zero count and Delta
    compared at the robust events; both sides' margins (threshold gap at the
    final Delta, final bracket) logged and consistent."""
    assert out["branch_hard"] == 0, f"{tag}: branching mismatch at event {out['first_branch_mismatch']}"
    np.testing.assert_array_equal(ev["m"], an.ev_m[:n_ev], err_msg=tag)
    rob = an.ev_robust[:n_ev] == 1
    np.testing.assert_array_equal(ev["status"][rob], an.ev_status[:n_ev][rob], err_msg=tag)
    np.testing.assert_array_equal(ev["z"][rob], an.ev_z[:n_ev][rob], err_msg=tag)
    done = rob & (ev["status"] == 0)
    np.testing.assert_allclose(ev["delta"][done], an.ev_delta[:n_ev][done], rtol=1e-9, err_msg=tag)
    if done.any():
        assert np.all(ev["gap"][done] > 0) and np.all(an.ev_gap[:n_ev][done] > 0), tag
        np.testing.assert_allclose(ev["bracket"][done], an.ev_bracket[:n_ev][done], rtol=1e-6, err_msg=tag)
    print(f"{tag} branching: {n_ev} events, near-ties {out['branch_near_ties']}, not robust "
          f"{int((an.ev_robust[:n_ev] == 0).sum())}, smallest gap GPU "
          f"{ev['gap'][done].min() if done.any() else float('nan'):.2e} oracle "
          f"{an.ev_gap[:n_ev][done].min() if done.any() else float('nan'):.2e}, bracket "
          f"{ev['bracket'][done].max() if done.any() else float('nan'):.2e}", flush=True)


def _same_or_near_tie(m_gpu, res, tag=""):
    """The GPU's multipliers of one event against the oracle's solve on the
    same residues: equal, or the oracle's outcome is not robust (near-tie).
    Returns the multipliers to continue with (the GPU's)."""
    if not np.array_equal(m_gpu, res["m"]):
        assert not res["robust"], f"{tag}: multipliers differ at a robust event"
        print(f"{tag}: branching near-tie adopted", flush=True)
    return m_gpu


def _anneal_lockstep(S, wl, n_walkers, seed, n_sweeps, sched_kw=None, mode=0, sigma=True, T=None, tpl=0):
    import torch
    gp, gs, op, osch = _pair(S, wl, n_walkers, seed, sched_kw, mode, sigma, T, tpl)
    an = O.Anneal(op, osch, n_walkers, seed)
    assert abs(gp.chi2_unit / an.chi2_unit - 1) < 1e-12
    gp.set_event_log(True)
    d, f = _trace_buffers(n_walkers, n_sweeps, wl.omega.size)
    gp.set_trace(0, n_sweeps, d.data_ptr(), f.data_ptr())
    gp.run(gs, 0, n_sweeps)
    torch.cuda.synchronize()
    g_d, g_f = d.cpu().numpy(), f.cpu().numpy()
    n_ev = n_sweeps // osch.branch_every
    ev = gp.read_events(n_ev, multipliers=True) if n_ev else None
    out = an.run(0, n_sweeps, trace=(0, n_sweeps), replay=g_f, replay_m=ev["m"] if n_ev else None)
    _check_trace(g_d, g_f, out)
    if n_ev:
        _check_branching(ev, an, out, n_ev, wl.name)
    chi2 = gp.read_chi2()
    np.testing.assert_allclose(chi2, an.chi2, rtol=1e-9)
    st = gp.read_state()
    np.testing.assert_allclose(st["a"], an.a, rtol=1e-9, atol=1e-12 * np.abs(an.a).max())
    np.testing.assert_allclose(st["F"], an.F, rtol=1e-12)
    spec = gp.read_spectrum()
    dw = wl.omega[1] - wl.omega[0]
    assert np.sum(np.abs(spec - an.mean_spectrum())) * dw <= 1e-10 * wl.m0
    _assert_untraced_twin(S, wl, n_walkers, seed, n_sweeps, gs, mode, sigma, gp, n_ev, tpl=tpl)
    return gp, an, out


def _assert_untraced_twin(S, wl, n_walkers, seed, n_sweeps, gs, mode, sigma, gp, n_ev, precision=0, tpl=0):
    """The same run without a trace window takes the kernel variant the
    benchmark times; its state, residues and branching log equal the traced
    (oracle-checked) run bit for bit."""
    tw = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma if sigma else None, wl.m0, wl.m1, mode)
    tw.set_tau_per_lane(tpl)
    tw.init_walkers(n_walkers, seed, precision=precision)
    tw.set_event_log(True)
    tw.run(gs, 0, n_sweeps)
    a, b = gp.read_state(), tw.read_state()
    for k in ("a", "F", "rate"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"untraced twin: {k}")
    np.testing.assert_array_equal(gp.read_chi2(), tw.read_chi2(), err_msg="untraced twin: chi2")
    if n_ev:
        ea, eb = gp.read_events(n_ev, multipliers=True), tw.read_events(n_ev, multipliers=True)
        for k in ("delta", "pr", "z", "status", "m"):
            np.testing.assert_array_equal(ea[k], eb[k], err_msg=f"untraced twin: events {k}")


def test_small_full_anneal_lockstep(S):
    """The small workload (64 bins, 32 times) end to end: 64 walkers x 2000 sweeps x 64 proposals, 20
    branching events; every proposal traced and compared."""
    wl = W.small_64x32()
    gp, an, out = _anneal_lockstep(S, wl, 64, wl.seed, wl.n_sweeps)
    assert out["proposals"] == 64 * 2000 * 64
    assert 0.2 < out["accepted"] / out["proposals"] < 0.8
    assert np.all(an.ev_status[:20] == 0)


@pytest.mark.parametrize("case", ["ragged", "bin_exact_unweighted", "single_tau", "two_walkers", "wide", "steep"])
def test_edge_shapes_lockstep(S, case):
    """Ragged walker counts and tau padding, the exact-bin kernel with the
    paper's unweighted residue, one tau point, the smallest population, the
    widest lane layout, and a steep kernel whose columns span the whole FP64
    range and underflow to zero (e^{-omega dtau} down to 1e-14 per step,
    e^{-omega tau} down to e^{-1000})."""
    rng = np.random.default_rng(77)
    tgt = W.Target([1.2, 3.0], [0.3, 0.6], [0.5, 0.5], 6.0)
    if case == "ragged":
        wl = W.make("r", 6.0, 50, W.uniform_tau(0.05, 1.5, 21), tgt, 1e-4, 3, 37, 300, 1e2, 1e-3, 50, 25, 5)
        kw, mode, sigma = dict(branch_every=50, resync_every=25), 0, True
    elif case == "bin_exact_unweighted":
        wl = W.make("b", 6.0, 40, W.uniform_tau(0.0, 2.0, 33), tgt, 1e-4, 4, 24, 200, 1e1, 1e-4, 100, 50, 6)
        kw, mode, sigma = dict(branch_every=100, resync_every=50), 1, False
    elif case == "single_tau":
        wl = W.make("s", 6.0, 16, np.array([0.4]), tgt, 1e-3, 5, 8, 100, 1e1, 1e-2, 50, 50, 7)
        kw, mode, sigma = dict(branch_every=50, resync_every=50, branch_fraction=0.25), 0, True
    elif case == "two_walkers":
        wl = W.make("t", 6.0, 24, W.uniform_tau(0.1, 1.0, 10), tgt, 1e-4, 6, 2, 100, 1e1, 1e-2, 50, 50, 8)
        kw, mode, sigma = dict(branch_every=50, resync_every=50, branch_fraction=0.5), 0, True
    elif case == "wide":
        wl = W.make("w", 20.0, 1024, W.uniform_tau(0.02, 3.0, 256), W.two_peak_random(rng, 20.0), 1e-5, 9, 48, 4,
                    1e3, 1e-2, 2, 1, 10, n_quad=20000)
        kw, mode, sigma = dict(branch_every=2, resync_every=1), 0, True
    else:
        steep = W.Target([5.0, 20.0], [2.0, 5.0], [0.5, 0.5], 100.0)
        wl = W.make("st", 100.0, 64, W.uniform_tau(0.02, 10.0, 32), steep, 1e-4, 11, 40, 200, 1e2, 1e-3, 100, 50, 12)
        kw, mode, sigma = dict(branch_every=100, resync_every=50), 0, True
    _anneal_lockstep(S, wl, wl.n_walkers, wl.seed, wl.n_sweeps, kw, mode, sigma)


@pytest.mark.parametrize("case", ["small", "three_chunks"])
def test_smoothing_lockstep(S, case):
    """Sec. 2.6 smoothing after every branching event (renormalised, F and
    chi^2 recomputed), every proposal traced against the oracle: the small
    workload (one 64-lane chunk per row), and 150 bins whose rows span three
    chunks with a ragged end (the value left of each chunk is carried)."""
    if case == "small":
        wl = W.small_64x32()
        _anneal_lockstep(S, wl, 64, wl.seed, 300, dict(smooth=0.05))
    else:
        tgt = W.Target([1.5, 4.0], [0.3, 0.8], [0.5, 0.5], 8.0)
        wl = W.make("sm", 8.0, 150, W.uniform_tau(0.05, 1.5, 24), tgt, 1e-4, 13, 20, 300, 1e2, 1e-3, 100, 50, 14)
        _anneal_lockstep(S, wl, wl.n_walkers, wl.seed, wl.n_sweeps, dict(branch_every=100, resync_every=50,
                                                                         smooth=0.2))


@pytest.mark.parametrize("smooth", [0.0, 0.01])
def test_adaptive_branching_lockstep(S, smooth):
    """Adaptive branching (fraction and imprint strength scaled by the mean
    running acceptance rate at each event), alone and with smoothing: the
    small workload end to end, every proposal, event and final state against
    the oracle (the mean is summed in a different order on each side; the
    zero-count targets agree unless f rho N lands within rounding of a half)."""
    wl = W.small_64x32()
    gp, an, out = _anneal_lockstep(S, wl, 64, wl.seed, wl.n_sweeps, dict(adaptive=1, smooth=smooth))
    z = an.ev_z[:20]
    assert np.all(an.ev_status[:20] == 0) and z[-1] < z[0]  # fewer walkers branched as acceptance falls


@pytest.mark.parametrize("adaptive", [0, 1])
def test_parallel_branch_search_lockstep(S, adaptive):
    """256 walkers, so every event runs the parallel Delta search: the small
    workload over 10 blocks, every proposal, event and final state against
    the oracle."""
    wl = W.small_64x32(n_sweeps=1000, n_walkers=256)
    gp, an, out = _anneal_lockstep(S, wl, 256, wl.seed, wl.n_sweeps, dict(adaptive=adaptive))
    assert np.all(an.ev_status[:10] == 0)


def test_self_cooling_lockstep(S):
    """Self-cooling (Sec. 2.4): the small workload over 20 blocks (2 boiling,
    5 cooling, 13 freezing), every proposal against the oracle, whose block
    temperatures come from the same residues in the same operation order."""
    wl = W.small_64x32()
    _anneal_lockstep(S, wl, 64, wl.seed, wl.n_sweeps, dict(self_cool=1, boil_blocks=2, cool_blocks=5))


def test_self_cooling_stages_and_refusal(S):
    """A self-cooling run split inside a block continues with that block's
    temperature (bits equal the one-call run); a run that starts inside a
    block no earlier call on the problem started is refused."""
    wl = W.small_64x32()
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, 400)
    sc = S.Schedule(T, self_cool=1, boil_blocks=1, cool_blocks=2)
    one = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    one.init_walkers(32, 3)
    one.run(sc, 0, 400)
    two = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    two.init_walkers(32, 3)
    two.run(sc, 0, 150)
    two.run(sc, 150, 250)
    np.testing.assert_array_equal(one.read_state()["a"], two.read_state()["a"])
    np.testing.assert_array_equal(one.read_chi2(), two.read_chi2())
    three = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    three.init_walkers(32, 3)
    with pytest.raises(S.SailError):
        three.run(sc, 150, 50)


@pytest.mark.parametrize("noise", ["none", "resampled"])
def test_paper_band_first_sweeps_lockstep(S, noise):
    """The paper's band (1000 bins, 64 times, 1500 walkers) under its
    protocol's schedule (self-cooling), exact data with the unweighted
    residue and resampled data with its standard errors: the first two
    sweeps of every walker against the oracle."""
    wl = W.paper_band(noise, n_seq=20000)
    _anneal_lockstep(S, wl, wl.n_walkers, wl.seed, 2,
                     dict(smooth=0.01, adaptive=1, self_cool=1, boil_blocks=20, cool_blocks=100),
                     sigma=wl.sigma is not None, T=np.ones(wl.n_sweeps))


@pytest.mark.parametrize("walk_len", [1, 4])
def test_selection_walk_lockstep(S, walk_len):
    """Sec. 2.3 index selection with a walk of independence Metropolis steps
    on a_j / A: the small workload, 64 walkers, 300 sweeps (three branching events),
    every proposal traced against the oracle (a different chosen pair would
    change the residue change far beyond the bar)."""
    wl = W.small_64x32()
    _anneal_lockstep(S, wl, 64, wl.seed, 300, dict(walk_len=walk_len))


def test_selection_walk_ragged_tail(S):
    """The walk with a bin count that leaves a partial last batch (no-op
    records past N_omega take no walk)."""
    tgt = W.Target([1.2, 3.0], [0.3, 0.6], [0.5, 0.5], 6.0)
    wl = W.make("rw", 6.0, 45, W.uniform_tau(0.05, 1.5, 19), tgt, 1e-4, 3, 21, 120, 1e2, 1e-3, 60, 30, 5)
    _anneal_lockstep(S, wl, wl.n_walkers, wl.seed, wl.n_sweeps, dict(branch_every=60, resync_every=30, walk_len=2))


def test_large_full_size_sampled_lockstep(S):
    """The large workload at full size (16384 walkers, 512 bins, 128 times) in the
    launch configuration the benchmark times: three traced sweeps, checked on
    a sample of walkers that the oracle replays one by one."""
    import torch
    wl = W.large_512x128()
    n = wl.n_walkers
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(n, wl.seed)
    gs = S.Schedule(T)
    ns = 3
    d, f = _trace_buffers(n, ns, wl.omega.size)
    gp.set_trace(0, ns, d.data_ptr(), f.data_ptr())
    gp.run(gs, 0, ns)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    ids = np.unique(np.concatenate([[0, 1, 7, 8, 63, 64, 4095, 8191, 16383], rng.choice(n, 23, replace=False)]))
    g_d, g_f = d[ids].cpu().numpy(), f[ids].cpu().numpy()
    del d, f
    op = O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    an = O.Anneal(op, O.Schedule(T), n, wl.seed, walker_ids=ids)
    assert abs(gp.chi2_unit / an.chi2_unit - 1) < 1e-12
    out = an.run(0, ns, trace=(0, ns), replay=g_f)
    _check_trace(g_d, g_f, out)
    st = gp.read_state()
    np.testing.assert_allclose(st["F"][ids], an.F, rtol=1e-12)
    np.testing.assert_allclose(st["a"][ids], an.a, rtol=1e-9, atol=1e-12 * np.abs(an.a).max())


def test_large_fp32_full_size_sampled_within_fp32_bar(S):
    """The FP32 loop at full size (16384 walkers, 512 bins, 128 times) in the
    launch configuration the benchmark times for it: three traced sweeps
    against the FP64 oracle on a sample of walkers, inside the FP32 bar
    (decisions within that band adopted by the oracle)."""
    import torch
    wl = W.large_512x128_fp32()
    n = wl.n_walkers
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(n, wl.seed, precision=S.SAIL_FP32)
    assert gp.layout() == (8, 16)
    ns = 3
    d, f = _trace_buffers(n, ns, wl.omega.size)
    gp.set_trace(0, ns, d.data_ptr(), f.data_ptr())
    gp.run(S.Schedule(T, resync_every=wl.resync_every), 0, ns)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    ids = np.unique(np.concatenate([[0, 1, 7, 8, 63, 64, 4095, 8191, 16383], rng.choice(n, 23, replace=False)]))
    g_d, g_f = d[ids].cpu().numpy(), f[ids].cpu().numpy()
    del d, f
    op = O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    an = O.Anneal(op, O.Schedule(T, resync_every=wl.resync_every), n, wl.seed, walker_ids=ids)
    out = an.run(0, ns, trace=(0, ns), replay=g_f, band=1e-5)
    assert out["hard_mismatch"] == 0, out["first_mismatch"]
    err = np.abs(g_d - out["dchi2"])
    worst = float(np.max(err / np.maximum(out["cond"], 1e-300)))
    print(f"worst |dchi2 error| / M over {err.size} proposals: {worst:.3e}", flush=True)
    assert np.all(err <= 1e-5 * out["cond"]), worst
    np.testing.assert_array_equal(g_f & 1, out["accept"] & 1)
    st = gp.read_state()
    np.testing.assert_allclose(st["a"][ids], an.a, rtol=1e-9, atol=1e-12 * np.abs(an.a).max())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_large_late_stage_sampled_lockstep(S, precision):
    """The large workload at full size (16384 walkers, 512 bins, 128 times)
    in the benchmark's launch configuration, late in the anneal: sweeps
    0-9899 run untraced (99 blocks with their resyncs and branching events,
    diverse spectra at low acceptance), then sweeps 9900-9902 run traced.
    A sample of 32 walkers is loaded into the oracle from the GPU state at
    sweep 9900 (spectra, reconstructions, residues, running rates, the
    residue unit) and replayed proposal by proposal: dchi^2 within 1e-12 M
    (FP64) or 1e-5 M (FP32 loop), identical accept bits apart from adopted
    near-ties, and the sample's state after the three sweeps.  A twin
    imported from the same checkpoint runs the three sweeps untraced and ends
    with the same bits as the traced run."""
    import torch
    fp32 = precision == "fp32"
    wl = W.large_512x128_fp32() if fp32 else W.large_512x128()
    prec = S.SAIL_FP32 if fp32 else S.SAIL_FP64
    n, k0, ns = wl.n_walkers, 9900, 3
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    gs = S.Schedule(T, resync_every=wl.resync_every)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(n, wl.seed, precision=prec)
    for b in range(k0 // 100):
        gp.run(gs, 100 * b, 100)
    st0, chi0 = gp.read_state(), gp.read_chi2()
    blob = gp.state_export()
    print(f"{precision}: sweep {k0}, median chi2/chi2_0 {np.median(chi0) / gp.chi2_unit:.3e}, "
          f"mean rate {st0['rate'].mean():.3f}", flush=True)
    d, f = _trace_buffers(n, ns, wl.omega.size)
    gp.set_trace(k0, k0 + ns, d.data_ptr(), f.data_ptr())
    gp.run(gs, k0, ns)
    torch.cuda.synchronize()
    gp.set_trace(0, 0)
    rng = np.random.default_rng(3)
    ids = np.unique(np.concatenate([[0, 1, 7, 8, 4095, 16383], rng.choice(n, 26, replace=False)]))
    g_d, g_f = d[ids].cpu().numpy(), f[ids].cpu().numpy()
    del d, f
    tw = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    tw.init_walkers(n, 1, precision=prec)
    tw.state_import(blob)
    tw.run(gs, k0, ns)
    st1, st_tw = gp.read_state(), tw.read_state()
    for key in ("a", "F", "rate"):
        np.testing.assert_array_equal(st1[key], st_tw[key], err_msg=f"untraced twin: {key}")
    np.testing.assert_array_equal(gp.read_chi2(), tw.read_chi2())
    op = O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    an = O.Anneal(op, O.Schedule(T, resync_every=wl.resync_every), n, wl.seed, walker_ids=ids)
    an.a[:] = st0["a"][ids]
    an.F[:] = st0["F"][ids]
    an.chi2[:] = chi0[ids]
    an.rate[:] = st0["rate"][ids]
    an.args.chi2_unit = gp.chi2_unit
    bar = 1e-5 if fp32 else 1e-12
    out = an.run(k0, k0 + ns, trace=(k0, k0 + ns), replay=g_f, band=bar)
    assert out["hard_mismatch"] == 0, out["first_mismatch"]
    err = np.abs(g_d - out["dchi2"])
    worst = float(np.max(err / np.maximum(out["cond"], 1e-300)))
    acc = float(np.mean(out["accept"] & 1))
    print(f"worst |dchi2 error| / M over {err.size} proposals: {worst:.3e}; acceptance {acc:.4f}; "
          f"near-ties {out['near_ties']}", flush=True)
    assert np.all(err <= bar * out["cond"]), worst
    np.testing.assert_array_equal(g_f & 1, out["accept"] & 1)
    np.testing.assert_allclose(st1["a"][ids], an.a, rtol=1e-9, atol=1e-12 * np.abs(an.a).max())
    np.testing.assert_allclose(st1["F"][ids], an.F, rtol=1e-5 if fp32 else 1e-12)


def test_large_full_size_branching_event(S):
    """The first branching event of the large workload at full size: the GPU's
    multipliers equal the oracle's solve on the same residues, and every
    target holds t a_donor + (1 - t) a_target afterwards."""
    wl = W.large_512x128()
    n = wl.n_walkers
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    runs = {}
    for name, be in (("plain", 10 ** 6), ("branch", 100)):
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.init_walkers(n, wl.seed)
        gp.set_event_log(True)
        gp.run(S.Schedule(T, branch_every=be), 0, 100)
        runs[name] = (gp, gp.read_chi2(), gp.read_state())
    chi2_pre, st_pre = runs["plain"][1], runs["plain"][2]
    gpb, _, st_post = runs["branch"]
    ev = gpb.read_events(1, multipliers=True)
    xi = O.branch_xi(wl.seed, 0, n)
    res = O.branch_solve(chi2_pre, xi, 0.25)
    assert res["status"] == 0 and ev["status"][0] == 0
    m = _same_or_near_tie(ev["m"][0], res, "large first event")
    if res["robust"]:
        assert ev["z"][0] == res["z"]
        assert abs(ev["delta"][0] / res["delta"] - 1) <= 1e-9
    print(f"large first event: gap GPU {ev['gap'][0]:.2e} oracle {res['gap']:.2e}, bracket GPU "
          f"{ev['bracket'][0]:.2e} oracle {res['bracket']:.2e}, robust {res['robust']}", flush=True)
    tg, dn = O.branch_pairs(m)
    t = 0.1
    expect = t * st_pre["a"][dn] + (1 - t) * st_pre["a"][tg]
    np.testing.assert_allclose(st_post["a"][tg], expect, rtol=1e-15, atol=0)
    keep = np.setdiff1d(np.arange(n), tg)
    np.testing.assert_array_equal(st_post["a"][keep], st_pre["a"][keep])


def test_large_full_size_protocol_event(S):
    """The first branching event of the large workload at full size under
    adaptive branching and smoothing (s = 0.01): the GPU's multipliers equal
    the oracle's solve at the fraction scaled by the mean of the GPU's rates,
    and every walker afterwards holds the renormalised smoothing of its
    spectrum after the imprint at the scaled strength."""
    wl = W.large_512x128()
    n = wl.n_walkers
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    runs = {}
    for name, be in (("plain", 10 ** 6), ("event", 100)):
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.init_walkers(n, wl.seed)
        gp.set_event_log(True)
        gp.run(S.Schedule(T, branch_every=be, adaptive=1, smooth=0.01), 0, 100)
        runs[name] = (gp, gp.read_chi2(), gp.read_state())
    chi2_pre, st_pre = runs["plain"][1], runs["plain"][2]
    gpe, _, st_post = runs["event"]
    ev = gpe.read_events(1, multipliers=True)
    rho = st_pre["rate"].mean()
    assert 0.0 < rho < 1.0
    res = O.branch_solve(chi2_pre, O.branch_xi(wl.seed, 0, n), 0.25 * rho)
    assert res["status"] == 0 and ev["status"][0] == 0
    tg, dn = O.branch_pairs(_same_or_near_tie(ev["m"][0], res, "large protocol event"))
    a = st_pre["a"].copy()
    t = 0.1 * rho
    a[tg] = t * st_pre["a"][dn] + (1 - t) * st_pre["a"][tg]
    prob = O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    rows = np.unique(np.concatenate([tg[:64], np.arange(0, n, 97)]))
    for l in rows:
        expect = O.renormalize(O.smooth(a[l], 0.01), wl.omega, prob.A, prob.B)
        np.testing.assert_allclose(st_post["a"][l], expect, rtol=1e-12, atol=1e-15 * expect.max())


@pytest.mark.parametrize("precision", [0, 1])
def test_deterministic_and_stageable(S, precision):
    """Two identical runs give identical bits, and a run split in stages at
    sweeps that are no resync boundary equals the run in one call (the state
    a launch leaves behind is all the next one needs)."""
    wl = W.small_64x32()
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    res = []
    for stages in ([(0, 370)], [(0, 370)], [(0, 37), (37, 163), (163, 370)]):
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.init_walkers(64, wl.seed, precision=precision)
        sched = S.Schedule(T)
        for k0, k1 in stages:
            gp.run(sched, k0, k1 - k0)
        st = gp.read_state()
        res.append((gp.read_chi2(), st["a"], st["F"], st["rate"]))
    for r in res[1:]:
        for x, y in zip(res[0], r):
            assert np.array_equal(x, y)


def test_staged_threshold_decides_like_the_fp64_log(S, monkeypatch):
    """The accept threshold is staged from an FP32 logarithm and retaken in
    FP64 inside its error band.  Forcing the FP64 retake for every decision
    (diagnostic switch) must give the same bits, and that path also runs in
    lockstep with the oracle."""
    wl = W.small_64x32()
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    res = []
    for exact in ("0", "1"):
        monkeypatch.setenv("SAIL_EXACT_THRESHOLD", exact)
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.init_walkers(64, wl.seed)
        gp.run(S.Schedule(T), 0, 300)
        st = gp.read_state()
        res.append((gp.read_chi2(), st["a"], st["F"], st["rate"]))
    for x, y in zip(*res):
        assert np.array_equal(x, y)
    monkeypatch.setenv("SAIL_EXACT_THRESHOLD", "1")
    _anneal_lockstep(S, wl, 64, wl.seed, 200)


def test_outputs_match_oracle_definitions(S):
    wl = W.small_64x32()
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(64, wl.seed)
    gp.run(S.Schedule(T), 0, 300)
    chi2 = gp.read_chi2()
    st = gp.read_state()
    np.testing.assert_allclose(gp.read_spectrum(), np.mean(st["a"], axis=0), rtol=1e-13)
    lo, hi = np.log10(chi2.min()), np.log10(chi2.max())
    h_auto = gp.read_chi2_hist(64)
    h_ref = O.chi2_hist(chi2, 64, lo, hi)
    np.testing.assert_array_equal(h_auto, h_ref)
    h2 = gp.read_chi2_hist(10, lo - 1, hi + 1)
    np.testing.assert_array_equal(h2, O.chi2_hist(chi2, 10, lo - 1, hi + 1))


def test_errors_leave_problem_usable(S):
    wl = W.small_64x32()
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    with pytest.raises(S.SailError):
        gp.run(S.Schedule(np.ones(10)), 0, 10)  # before init
    gp.init_walkers(8, 1)
    with pytest.raises(S.SailError):
        gp.run(S.Schedule(np.ones(10)), 5, 10)  # past the schedule
    with pytest.raises(S.SailError):
        gp.run(S.Schedule(np.ones(10), branch_every=30, resync_every=7), 0, 10)
    with pytest.raises(S.SailError):
        gp.run(S.Schedule(np.ones(10), eps0=1.5), 0, 10)
    with pytest.raises(S.SailError):
        gp.run(S.Schedule(np.full(10, -1.0)), 0, 10)
    gp.run(S.Schedule(np.ones(10)), 0, 10)
    assert np.all(np.isfinite(gp.read_chi2()))


@pytest.mark.parametrize("tau_per_lane", [8, 16, 32])
def test_fp32_loop_first_sweeps_within_fp32_bar(S, tau_per_lane):
    """FP32 residual loop (the variant the large FP32 workload runs): every proposal of the first two
    sweeps against the FP64 oracle, in every FP32 lane layout.  The loop
    carries Phi and the columns in FP32, so the bar is
    (TPL + log2 L + 8) u_32 M <= 1e-5 M; decisions whose margin falls inside
    that band are adopted by the oracle."""
    import torch
    wl = W.small_64x32()
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.set_tau_per_lane(tau_per_lane)
    gp.init_walkers(64, wl.seed, precision=S.SAIL_FP32)
    lanes, tpl = gp.layout()
    assert tpl == tau_per_lane and lanes * tpl == 32
    ns = 2
    d, f = _trace_buffers(64, ns, wl.omega.size)
    gp.set_trace(0, ns, d.data_ptr(), f.data_ptr())
    gp.run(S.Schedule(T), 0, ns)
    torch.cuda.synchronize()
    g_d, g_f = d.cpu().numpy(), f.cpu().numpy()
    an = O.Anneal(O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1), O.Schedule(T), 64, wl.seed)
    out = an.run(0, ns, trace=(0, ns), replay=g_f, band=1e-5)
    assert out["hard_mismatch"] == 0, out["first_mismatch"]
    err = np.abs(g_d - out["dchi2"])
    assert np.all(err <= 1e-5 * out["cond"]), np.max(err / out["cond"])
    np.testing.assert_array_equal(g_f & 1, out["accept"] & 1)


def test_fp32_anneal_quality_against_fp64(S):
    """A whole anneal of the small workload with the FP32 loop (FP64 resync every 50 sweeps)
    lands in the same residue range as the FP64 path, and the FP64 resync keeps
    both sum rules to rounding."""
    wl = W.small_64x32()
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    res = {}
    for prec, rs in ((S.SAIL_FP64, 100), (S.SAIL_FP32, 50)):
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.init_walkers(64, wl.seed, precision=prec)
        gp.run(S.Schedule(T, resync_every=rs), 0, wl.n_sweeps)
        res[prec] = (gp.read_chi2() / gp.chi2_unit, gp.read_state()["a"], gp.read_spectrum())
    c64, a64, s64 = res[S.SAIL_FP64]
    c32, a32, s32 = res[S.SAIL_FP32]
    assert 0.3 < np.median(c32) / np.median(c64) < 3.0
    dw = wl.omega[1] - wl.omega[0]
    A, B = wl.m0 / dw, wl.m1 / dw
    assert np.max(np.abs(a32.sum(axis=1) - A)) <= 1e-12 * A
    assert np.max(np.abs((a32 * wl.omega).sum(axis=1) - B)) <= 1e-12 * B
    assert np.sum(np.abs(s32 - s64)) * dw < 0.5


def test_fp32_anneal_within_the_oracles_seed_spread(S):
    """Whole anneals of the small workload, statistically: the FP32 loop's
    final median residue and averaged spectrum lie within 3x the FP64
    oracle's own seed-to-seed spread of an ensemble of six other seeds (the
    median within 3 standard deviations of the ensemble mean, the spectrum
    within 3x the largest distance of an ensemble member from the ensemble
    mean, in L1), and both sum rules hold to rounding."""
    wl = W.small_64x32()
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    dw = wl.omega[1] - wl.omega[0]
    op = O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    med, spec = [], []
    for sd in range(wl.seed + 1000, wl.seed + 1006):
        an = O.Anneal(op, O.Schedule(T), 64, sd)
        an.run(0, wl.n_sweeps)
        med.append(float(np.median(an.chi2 / an.chi2_unit)))
        spec.append(an.mean_spectrum())
    med, spec = np.array(med), np.array(spec)
    centre = spec.mean(axis=0)
    l1_members = np.array([np.sum(np.abs(s - centre)) * dw for s in spec])
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(64, wl.seed, precision=S.SAIL_FP32)
    gp.run(S.Schedule(T, resync_every=50), 0, wl.n_sweeps)
    m32 = float(np.median(gp.read_chi2() / gp.chi2_unit))
    l1_32 = float(np.sum(np.abs(gp.read_spectrum() - centre)) * dw)
    print(f"oracle medians {np.round(med, 6)} (sd {med.std(ddof=1):.3g}); FP32 {m32:.6g}; spectrum L1 from the "
          f"ensemble mean: members up to {l1_members.max():.3g}, FP32 {l1_32:.3g}", flush=True)
    assert med.std(ddof=1) > 0
    assert abs(m32 - med.mean()) <= 3.0 * med.std(ddof=1)
    assert l1_32 <= 3.0 * l1_members.max()
    a = gp.read_state()["a"]
    A, B = wl.m0 / dw, wl.m1 / dw
    assert np.max(np.abs(a.sum(axis=1) - A)) <= 1e-12 * A
    assert np.max(np.abs((a * wl.omega).sum(axis=1) - B)) <= 1e-12 * B


def test_checkpoint_resume_is_bit_exact(S):
    """Export after 250 sweeps, destroy, import into a fresh problem and
    continue: identical bits to the uninterrupted run (counter-based stream)."""
    wl = W.small_64x32()
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    ref = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    ref.init_walkers(64, wl.seed)
    ref.run(S.Schedule(T), 0, 500)
    a = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    a.init_walkers(64, wl.seed)
    a.run(S.Schedule(T), 0, 250)
    blob = a.state_export()
    a.close()
    b = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    b.init_walkers(64, 999)
    b.state_import(blob)
    b.run(S.Schedule(T), 250, 250)
    assert np.array_equal(ref.read_chi2(), b.read_chi2())
    ra, rb = ref.read_state(), b.read_state()
    assert np.array_equal(ra["a"], rb["a"]) and np.array_equal(ra["F"], rb["F"])
    with pytest.raises(S.SailError):
        c = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        c.init_walkers(32, 1)
        c.state_import(blob)


def test_watchdog_detects_and_rolls_back(S):
    """Failure detection, forced from the host.  With the watchdog on and a
    loose bound the anneal has the bits of a run without it.  A bound below
    any real drift (1e-300) trips at the first resync of the next call
    (sweep 225), which then returns SAIL_ENUMERIC with the walkers restored
    bit for bit to their state at the call's start (sweep 200); rerun with
    the loose bound, the call continues exactly like the unwatched run.  A
    checkpoint whose spectrum holds a NaN (planted on the host) trips the
    non-finite check at its first resync and is restored as imported."""
    wl = W.small_64x32(n_sweeps=600, n_walkers=32)
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    sc = S.Schedule(T, branch_every=100, resync_every=25)
    ref = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    ref.init_walkers(32, wl.seed)
    ref.run(sc, 0, 200)
    ref_200 = ref.read_state()
    ref.run(sc, 200, 100)
    ref_300, ref_chi2_300 = ref.read_state(), ref.read_chi2()
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(32, wl.seed)
    with pytest.raises(S.SailError) as e:
        gp.set_watchdog(-1.0)
    assert e.value.status == 1
    gp.set_watchdog(1e-6)
    gp.run(sc, 0, 200)
    assert gp.watchdog_report() == (-1, -1)
    st = gp.read_state()
    for k in ("a", "F", "rate"):
        np.testing.assert_array_equal(st[k], ref_200[k], err_msg=k)
    gp.set_watchdog(1e-300)
    with pytest.raises(S.SailError) as e:
        gp.run(sc, 200, 100)
    assert e.value.status == 5 and "drift" in str(e.value), str(e.value)
    assert gp.watchdog_report() == (225, 200)
    st = gp.read_state()
    for k in ("a", "F", "rate"):
        np.testing.assert_array_equal(st[k], ref_200[k], err_msg=f"rolled back {k}")
    gp.set_watchdog(1e-6)
    gp.run(sc, 200, 100)
    st = gp.read_state()
    for k in ("a", "F", "rate"):
        np.testing.assert_array_equal(st[k], ref_300[k], err_msg=f"resumed {k}")
    np.testing.assert_array_equal(gp.read_chi2(), ref_chi2_300)
    # a non-finite spectrum value planted in a checkpoint
    blob = bytearray(gp.state_export())
    header = 48
    l, j = 5, 17
    off = header + 8 * (l * wl.omega.size + j)
    blob[off:off + 8] = np.array([np.nan]).tobytes()
    gp.state_import(bytes(blob))
    planted = gp.read_state()
    with pytest.raises(S.SailError) as e:
        gp.run(sc, 300, 100)
    assert e.value.status == 5 and "non-finite" in str(e.value), str(e.value)
    assert gp.watchdog_report() == (325, 300)
    st = gp.read_state()
    np.testing.assert_array_equal(st["a"], planted["a"])  # NaN compares equal at the same place
    assert np.isnan(st["a"][l, j]) and np.isfinite(np.delete(st["a"].ravel(), l * wl.omega.size + j)).all()


@pytest.mark.parametrize("i", range(16))
def test_random_shapes_lockstep(S, i):
    """Seeded random shapes and protocols in lockstep with the oracle, every
    proposal traced, over every branching event of the run."""
    wl, kw, mode, sigma = _random_case(i)
    print(f"case {i}: {wl.omega.size} bins, {wl.tau.size} times, {wl.n_walkers} walkers, {wl.n_sweeps} sweeps, "
          f"mode {mode}, weighted {sigma}, {kw}", flush=True)
    _anneal_lockstep(S, wl, wl.n_walkers, wl.seed, wl.n_sweeps, kw, mode, sigma)


@pytest.mark.parametrize("i,tpl", [(0, 4), (3, 4), (5, 4), (6, 4), (8, 8), (12, 4), (14, 4), (15, 8), (3, 8)])
def test_random_shapes_lockstep_small_tiles(S, i, tpl):
    """The smaller FP64 tiles (4 and 8 tau points per lane: more lanes per
    walker, a longer reduction) on random shapes and protocols spanning 2 to
    64 lanes, in lockstep with the oracle over every branching event, as at
    the default tile."""
    wl, kw, mode, sigma = _random_case(i)
    print(f"case {i}, {tpl} tau per lane: {wl.omega.size} bins, {wl.tau.size} times, {wl.n_walkers} walkers, "
          f"{wl.n_sweeps} sweeps, mode {mode}, weighted {sigma}, {kw}", flush=True)
    gp, _, _ = _anneal_lockstep(S, wl, wl.n_walkers, wl.seed, wl.n_sweeps, kw, mode, sigma, tpl=tpl)
    lanes, got = gp.layout()
    assert got == tpl or (got > tpl and lanes == 64), (lanes, got)


@pytest.mark.parametrize("i", range(0, 16, 2))
def test_random_shapes_fp32_first_sweeps(S, i):
    """The FP32 loop on the same random shapes and protocols: every proposal
    of the first two sweeps against the FP64 oracle at the FP32 bar (1e-5 M,
    decisions inside that band adopted by the oracle)."""
    import torch
    wl, kw, mode, sigma = _random_case(i)
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
    sg = wl.sigma if sigma else None
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, sg, wl.m0, wl.m1, mode)
    gp.init_walkers(wl.n_walkers, wl.seed, precision=S.SAIL_FP32)
    print(f"case {i}: {wl.omega.size} bins, {wl.tau.size} times, {wl.n_walkers} walkers, layout {gp.layout()}",
          flush=True)
    ns = 2
    d, f = _trace_buffers(wl.n_walkers, ns, wl.omega.size)
    gp.set_trace(0, ns, d.data_ptr(), f.data_ptr())
    gp.run(S.Schedule(T, **kw), 0, ns)
    torch.cuda.synchronize()
    g_d, g_f = d.cpu().numpy(), f.cpu().numpy()
    an = O.Anneal(O.Problem(wl.omega, wl.tau, wl.Ft, sg, wl.m0, wl.m1, mode), O.Schedule(T, **kw),
                  wl.n_walkers, wl.seed)
    out = an.run(0, ns, trace=(0, ns), replay=g_f, band=1e-5)
    assert out["hard_mismatch"] == 0, out["first_mismatch"]
    err = np.abs(g_d - out["dchi2"])
    worst = float(np.max(err / np.maximum(out["cond"], 1e-300)))
    print(f"worst |dchi2 error| / M over {err.size} proposals: {worst:.3e}", flush=True)
    assert np.all(err <= 1e-5 * out["cond"]), worst
    np.testing.assert_array_equal(g_f & 1, out["accept"] & 1)


@pytest.mark.parametrize("case", ["max_bins", "max_lanes"])
def test_maximum_sizes_lockstep(S, case):
    """The largest shapes the layout takes, in lockstep with the oracle: the
    most bins one workgroup's LDS holds (N_omega = 2556, 16 tau points) and
    the widest lane layout, 64 lanes of 16 tau points for one walker per
    wavefront (N_tau = 1024, the FP64 limit), each over a branching event."""
    tgt = W.Target([1.2, 3.0], [0.3, 0.6], [0.5, 0.5], 6.0)
    if case == "max_bins":
        wl = W.make("mb", 6.0, 2556, W.uniform_tau(0.05, 1.5, 16), tgt, 1e-4, 13, 12, 4, 1e2, 1e-3, 2, 1, 14,
                    n_quad=40000)
    else:
        wl = W.make("ml", 6.0, 48, W.uniform_tau(0.01, 4.0, 1024), tgt, 1e-4, 15, 6, 4, 1e2, 1e-3, 2, 1, 16)
    gp, an, out = _anneal_lockstep(S, wl, wl.n_walkers, wl.seed, wl.n_sweeps, dict(branch_every=2, resync_every=1))
    lanes, tpl = gp.layout()
    assert (lanes, tpl) == ((1, 16) if case == "max_bins" else (64, 16))


def test_fp32_widest_layout_within_fp32_bar(S):
    """FP32 at the largest time grid (N_tau = 1024: 32 lanes of 32 tau points,
    two walkers per wavefront): every proposal of two sweeps against the FP64
    oracle at 1e-5 M."""
    import torch
    tgt = W.Target([1.2, 3.0], [0.3, 0.6], [0.5, 0.5], 6.0)
    wl = W.make("f32w", 6.0, 32, W.uniform_tau(0.01, 6.0, 1024), tgt, 1e-4, 17, 4, 2, 1e2, 1e-3, 100, 100, 18)
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, 100)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.set_tau_per_lane(32)
    gp.init_walkers(4, wl.seed, precision=S.SAIL_FP32)
    assert gp.layout() == (32, 32)
    d, f = _trace_buffers(4, 2, wl.omega.size)
    gp.set_trace(0, 2, d.data_ptr(), f.data_ptr())
    gp.run(S.Schedule(T), 0, 2)
    torch.cuda.synchronize()
    g_d, g_f = d.cpu().numpy(), f.cpu().numpy()
    an = O.Anneal(O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1), O.Schedule(T), 4, wl.seed)
    out = an.run(0, 2, trace=(0, 2), replay=g_f, band=1e-5)
    assert out["hard_mismatch"] == 0, out["first_mismatch"]
    err = np.abs(g_d - out["dchi2"])
    print(f"FP32 N_tau 1024: worst |dchi2 error| / M {np.max(err / out['cond']):.3e}", flush=True)
    assert np.all(err <= 1e-5 * out["cond"])
    np.testing.assert_array_equal(g_f & 1, out["accept"] & 1)


def test_sizes_beyond_the_layout_are_refused(S):
    """One tau point past the widest layout, and one walker past what the
    branching workgroup covers, are refused with SAIL_EINVAL before any
    sweep runs; a refused run leaves the problem usable."""
    om = W.bin_centres(6.0, 16)
    tau = W.uniform_tau(0.01, 6.0, 1025)
    F = np.exp(-np.outer(tau, om)).sum(axis=1)
    with pytest.raises(S.SailError) as e:
        S.Problem(om, tau, F, None, 1.0, 3.0)
    assert e.value.status == 1 and "n_tau" in str(e.value)
    tau = W.uniform_tau(0.05, 1.5, 8)
    F = np.exp(-np.outer(tau, om)).sum(axis=1)
    gp = S.Problem(om, tau, F, None, 1.0, 3.0)
    gp.init_walkers(16385, 1)
    with pytest.raises(S.SailError) as e:
        gp.run(S.Schedule(np.ones(10)), 0, 1)
    assert e.value.status == 1 and "walkers" in str(e.value)
    gp.init_walkers(16384, 1)
    gp.run(S.Schedule(np.ones(10)), 0, 1)
