"""Benchmark: walker proposals per second of the annealing hot path.

One step = one block of the anneal on one GPU: 100 sweeps of every walker
(each sweep N_omega proposals: Philox draws, sum-rule move, incremental
residual loop over all tau, reduction, Metropolis accept), the exact resync
of every walker, and one imprinted-branching event (solve, imprint,
recompute of the targets).  The default workload is the production-scale
FP64 configuration: 512 bins on [0, 20], 128 times on [0.02, 3], 16384
walkers, 20000 sweeps (200 steps), double-Lorentzian synthetic data with
1e-5 relative noise.  Inputs are resident in HBM before timing starts.

Prints one JSON line: the metric, the roofline
of the sweep kernel from HIP events on its launch stream, and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector
SWEEPS_PER_STEP = 100
# workload -> stem of its sweep-kernel summaries under profiles/
WORKLOADS = {"fp64": "k_sweep_fp64_512x128x16384", "fp32": "k_sweep_fp32_512x128x16384",
             "batched": "k_sweep_batched_fp32_256jobs", "served": None, "band": None}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed blocks of 100 sweeps (200 = the whole anneal)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fp64", choices=list(WORKLOADS),
                    help="fp64: 512 x 128 x 16384 walkers, FP64 loop (default); fp32: the same with the FP32 loop "
                         "and FP64 resync every 50 sweeps; batched: 256 mixed-size FP32 jobs in shared launches "
                         "(a step is one round of 50 sweeps); served: Poisson stream of such jobs into the server; "
                         "band: the paper's Lorentzian band with its protocol (self-cooling, smoothing, adaptive "
                         "branching), reporting the skew")
    ap.add_argument("--band-noise", default="none", choices=["none", "iid", "resampled"],
                    help="band: exact data, iid noise of --level, or the resampled generator with --n-seq sequences")
    ap.add_argument("--level", type=float, default=1e-4, help="band: iid noise level")
    ap.add_argument("--n-seq", type=int, default=20000, help="band: sequences of the resampled generator")
    ap.add_argument("--band-sweeps", type=int, default=20000,
                    help="band: length of the anneal in sweeps (the band line always runs the whole anneal)")
    ap.add_argument("--band-cool", type=int, default=100, help="band: cooling blocks of the self-cooling schedule")
    ap.add_argument("--rate", type=float, default=50.0, help="served: offered load, jobs/s")
    ap.add_argument("--duration", type=float, default=30.0, help="served: arrival window, s")
    ap.add_argument("--max-jobs", type=int, default=256, help="served: in-flight jobs at most")
    ap.add_argument("--jobs", type=int, default=256, help="batched: number of jobs")
    ap.add_argument("--smooth", type=float, default=0.0,
                    help="fp64/fp32: smoothing amplitude of Sec. 2.6 after every branching event (paper: 0.01)")
    ap.add_argument("--adaptive", action="store_true",
                    help="fp64/fp32: adaptive branching (fraction and imprint scaled by the mean acceptance rate)")
    ap.add_argument("--self-cool", default="",
                    help="fp64/fp32: self-cooling of Sec. 2.4 as 'boil_blocks,cool_blocks' (blocks of 100 sweeps)")
    ap.add_argument("--tpl", type=int, default=0,
                    help="fp64/fp32: tau points per lane (0: the library's choice; FP64 8 or 16, FP32 16 or 32)")
    ap.add_argument("--cpu-sample-walkers", type=int, default=4096)
    ap.add_argument("--cpu-sample-sweeps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-finish", action="store_true",
                    help="fp64/fp32: skip the untimed rest of the anneal (final chi2 then stays unmeasured)")
    ap.add_argument("--no-precision-match", action="store_true",
                    help="fp64: skip the untimed FP32-loop anneal on the same seeds")
    ap.add_argument("--no-extras", action="store_true",
                    help="fp64: skip the batched and served measurements appended to the line")
    ap.add_argument("--extras-rate", type=float, default=15.0, help="fp64 line's served measurement: jobs/s")
    ap.add_argument("--extras-duration", type=float, default=20.0, help="fp64 line's served measurement: window, s")
    ap.add_argument("--plain-jobs", type=int, default=4,
                    help="batched/served: jobs solved one at a time on the plain FP64 path for comparison")
    return ap.parse_args()


def cpu_model() -> str:
    """The host CPU's model name (Linux), or the platform's description."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def matched(median_a: float, median_b: float, rel: float = 0.05) -> bool:
    """Final residues match when the medians agree within rel (5%)."""
    return abs(median_a / median_b - 1.0) <= rel


def sweep_source_digest() -> str:
    """sha256 prefix of the sweep kernel's source: sail.hip from its start to
    the end of k_sweep_batched (the helpers, the sweep and its wrappers)."""
    import hashlib
    text = open(os.path.join(ROOT, "paper_1609_07936_amd", "csrc", "sail.hip"), "rb").read()
    i = text.index(b"void k_sweep_batched(")
    j = text.index(b"\n}\n", i) + 3
    return hashlib.sha256(text[:j]).hexdigest()[:16]


def measured_lds(workload: str, avg_launch_ms: float):
    """LDS bytes per sweep launch (read + written) from the committed LDS
    counter summary, with the probe's measured LDS read ceiling, if it was
    taken on the sweep kernel's source as it stands (else None)."""
    col = {"fp64": 0, "fp32": 1}.get(workload)
    path = os.path.join(ROOT, "profiles", "lds_bandwidth_and_sweep_lds_counters.md")
    if col is None or not os.path.exists(path):
        return None
    text = open(path).read()
    digest = ceiling = None
    rows = {}
    for line in text.splitlines():
        if line.startswith("sweep_source_sha256_16:"):
            digest = line.split(":", 1)[1].strip()
        elif line.startswith("Ceiling used below:"):
            ceiling = float(line.split(":", 1)[1].split("TB/s")[0])
        elif line.startswith("| LDS bytes"):
            cells = [c.strip() for c in line.strip("|").split("|")]
            rows[cells[0]] = float(cells[1 + col])
    if digest != sweep_source_digest() or ceiling is None or len(rows) < 2:
        return None
    total = rows["LDS bytes read per launch"] + rows["LDS bytes written per launch"]
    tbs = total / (avg_launch_ms * 1e-3) / 1e12
    return {"bytes_per_launch": total, "achieved": tbs, "ceiling": ceiling, "unit": "TB/s", "frac": tbs / ceiling}


def measured_traffic(workload: str):
    """HBM bytes per sweep launch from the committed FETCH_SIZE / WRITE_SIZE
    summary, if it was taken on the sweep kernel's source as it stands (else
    None)."""
    if WORKLOADS[workload] is None:
        return None
    path = os.path.join(ROOT, "profiles", f"{WORKLOADS[workload]}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "|", "#")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("sweep_source_sha256_16") != sweep_source_digest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def fp64_comparison(S, W, wl, T, gp32, chi2_32, value32, stream, smooth=0.0, adaptive=0) -> dict:
    """The FP32-loop anneal against the FP64 path (the FP64 GPU path is
    parity-tested against the CPU oracle; the oracle itself would take hours
    at this size): the same walkers, seeds and schedule with resync every 100
    sweeps, run after the timed region.  Reports the L1 distance of the
    averaged spectra (against a unit zeroth moment), the ratio of the median
    final residues, the FP32 path's largest sum-rule drift over the walkers,
    and its proposals/s against the FP64 path's."""
    import torch
    fp64_wl = W.large_512x128()
    sp32 = gp32.read_spectrum(stream=stream)
    a32 = gp32.read_state(stream=stream)["a"]
    dw = wl.omega[1] - wl.omega[0]
    A, B = wl.m0 / dw, wl.m1 / dw
    drift = max(float(np.max(np.abs(a32.sum(axis=1) - A)) / A),
                float(np.max(np.abs((a32 * wl.omega).sum(axis=1) - B)) / B))
    del a32
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(wl.n_walkers, wl.seed, precision=S.SAIL_FP64, stream=stream)
    sched = S.Schedule(T, branch_every=SWEEPS_PER_STEP, resync_every=fp64_wl.resync_every, smooth=smooth,
                       adaptive=adaptive)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(wl.n_sweeps // SWEEPS_PER_STEP):
        gp.run(sched, s * SWEEPS_PER_STEP, SWEEPS_PER_STEP, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sp64 = gp.read_spectrum(stream=stream)
    chi2_64 = gp.read_chi2(stream=stream)
    return {"spectrum_L1": float(np.sum(np.abs(sp32 - sp64)) * dw / wl.m0),
            "median_chi2_ratio_fp32_over_fp64": float(np.median(chi2_32) / np.median(chi2_64)),
            "matched_final_chi2": matched(float(np.median(chi2_32)), float(np.median(chi2_64))),
            "sum_rule_drift_max_fp32": drift,
            "fp64_proposals_per_s": wl.n_walkers * wl.omega.size * wl.n_sweeps / dt,
            "speedup_fp32_over_fp64": value32 / (wl.n_walkers * wl.omega.size * wl.n_sweeps / dt)}


def fp32_match(S, W, gp64, chi2_64, sched64, stream) -> dict:
    """The FP32-loop path (FP64 resync and renormalisation every 50 sweeps) on
    the same data, seeds and schedule, run untimed after the FP64 anneal:
    its final residues against the FP64 path's (matched when the medians
    agree within 5%) and the L1 distance of the averaged spectra."""
    import torch
    wl = W.large_512x128_fp32()
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    gp.init_walkers(wl.n_walkers, wl.seed, precision=S.SAIL_FP32, stream=stream)
    c = sched64.c
    sched = S.Schedule(sched64.T, branch_every=c.branch_every, resync_every=wl.resync_every, smooth=c.smooth,
                       adaptive=c.adaptive, self_cool=c.self_cool, boil_blocks=c.boil_blocks,
                       cool_blocks=c.cool_blocks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(wl.n_sweeps // SWEEPS_PER_STEP):
        gp.run(sched, s * SWEEPS_PER_STEP, SWEEPS_PER_STEP, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    chi2_32 = gp.read_chi2(stream=stream)
    dw = wl.omega[1] - wl.omega[0]
    l1 = float(np.sum(np.abs(gp.read_spectrum(stream=stream) - gp64.read_spectrum(stream=stream))) * dw / wl.m0)
    m32, m64 = float(np.median(chi2_32)), float(np.median(chi2_64))
    return {"fp32_final_chi2_over_chi2_0_median": m32 / gp.chi2_unit,
            "fp32_final_chi2_over_chi2_0_min": float(chi2_32.min()) / gp.chi2_unit,
            "median_final_chi2_ratio_fp32_over_fp64": m32 / m64,
            "matched_final_chi2": matched(m32, m64),
            "spectrum_L1_fp32_vs_fp64": l1,
            "fp32_proposals_per_s_untimed_run": wl.n_walkers * wl.omega.size * wl.n_sweeps / dt}


def cpu_baseline(wl, T, n_walkers, n_sweeps, one_thread_walkers=0) -> dict:
    """The oracle on a walker sample of the workload, all host threads; with
    one_thread_walkers > 0 also a smaller sample on one thread."""
    import oracle as O
    op = O.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)

    def sample(nw):
        stride = max(1, wl.n_walkers // nw)
        ids = np.arange(0, wl.n_walkers, stride)[:nw]
        # sweeps only: the sample's walkers are a subset, so no resync or branching
        an = O.Anneal(op, O.Schedule(T, branch_every=10 ** 6, resync_every=10 ** 6), wl.n_walkers, wl.seed,
                      walker_ids=ids)
        t0 = time.perf_counter()
        out = an.run(0, n_sweeps)
        return ids.size, stride, out["proposals"], time.perf_counter() - t0

    threads = O.max_threads()
    nw, stride, props, dt = sample(n_walkers)
    res = {"value": props / dt, "unit": "proposals/s", "cores": threads, "cpu_model": cpu_model(), "kind": "oracle",
           "sample": f"{nw} of {wl.n_walkers} walkers (every {stride}th), sweeps 0-{n_sweeps - 1} of the same "
                     f"schedule (sweeps only, no resync or branching): {props} proposals in {dt:.2f} s"}
    if one_thread_walkers > 0:
        O.set_threads(1)
        nw1, _, props1, dt1 = sample(one_thread_walkers)
        O.set_threads(threads)
        res["value_1_thread"] = props1 / dt1
        res["sample_1_thread"] = f"{nw1} walkers, sweeps 0-{n_sweeps - 1}: {props1} proposals in {dt1:.2f} s"
    return res


def plain_fp64_solves(S, W, jobs, scheds) -> dict:
    """The comparison path for batches and the server: the same jobs solved
    one at a time on the plain one-instance FP64 path (sail_run_schedule on
    each problem alone, walkers initialised inside the clock), with their
    final median residues."""
    import torch
    times, rel, prop = [], [], 0
    for wl, sc in zip(jobs, scheds):
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.autotune_layout(wl.n_walkers, S.SAIL_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gp.init_walkers(wl.n_walkers, wl.seed, precision=S.SAIL_FP64)
        gp.run(sc, 0, wl.n_sweeps)
        chi2 = gp.read_chi2()
        times.append(time.perf_counter() - t0)
        rel.append(float(np.median(chi2) / gp.chi2_unit))
        prop += wl.n_walkers * wl.omega.size * wl.n_sweeps
    return {"jobs": len(jobs), "solve_s": times, "solves_per_s": len(times) / sum(times),
            "proposals_per_s": prop / sum(times), "final_chi2_over_chi2_0_median": rel}


def batched(args):
    print(json.dumps(batched_line(args)), flush=True)


def batched_line(args) -> dict:
    """256 independent inversions of mixed sizes (N_omega in
    {128..1024}, N_tau in {32..256}, walkers in {256, 1024, 4096}), FP32 loop
    with FP64 resync every 50 sweeps, 1000 sweeps each, branching every 100;
    every round is one shared sweep launch plus shared resync / branch
    launches.  A step is one round (50 sweeps of every job)."""
    import torch
    from paper_1609_07936_amd import sail as S
    from paper_1609_07936_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    jobs = W.batch_jobs(args.jobs)
    per_step = jobs[0].resync_every
    n_sweeps = jobs[0].n_sweeps
    steps = args.steps if args.steps * per_step <= n_sweeps else n_sweeps // per_step
    warm = args.warmup
    stream = torch.cuda.current_stream()
    probs, scheds = [], []
    t_tune = time.perf_counter()
    for wl in jobs:
        gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
        gp.autotune_layout(wl.n_walkers, S.SAIL_FP32, stream=stream)
        probs.append(gp)
        scheds.append(S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), branch_every=wl.branch_every,
                                 resync_every=wl.resync_every))
    t_tune = time.perf_counter() - t_tune
    batch = S.Batch(probs)

    def init():
        for gp, wl in zip(probs, jobs):
            gp.init_walkers(wl.n_walkers, wl.seed, precision=S.SAIL_FP32, stream=stream)

    init()
    for s in range(warm):
        batch.run(scheds, s * per_step, per_step, stream=stream)
    init()
    batch.run(scheds, 0, 0, stream=stream)  # uploads the schedules outside the timed region
    batch.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        batch.run(scheds, s * per_step, per_step, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sweep_ms, launches = batch.sweep_timing(reset=True)
    swept = steps * per_step
    proposals = sum(wl.n_walkers * wl.omega.size for wl in jobs) * swept
    flops = 8.0 * sum(wl.n_walkers * wl.omega.size * wl.tau.size for wl in jobs) * swept
    achieved = flops / (sweep_ms * 1e-3) / 1e12
    rel = np.array([np.median(gp.read_chi2(stream=stream)) / gp.chi2_unit for gp in probs])
    plain = None
    if args.plain_jobs > 0 and steps * per_step == n_sweeps:
        k = min(args.plain_jobs, len(jobs))
        plain = plain_fp64_solves(S, W, jobs[:k], scheds[:k])
        plain["median_final_chi2_ratio_batched_over_plain"] = [float(a / b) for a, b in
                                                                zip(rel[:k], plain["final_chi2_over_chi2_0_median"])]
        plain["matched_final_chi2"] = all(matched(a, b) for a, b in zip(rel[:k], plain["final_chi2_over_chi2_0_median"]))
    layouts = {}
    for gp in probs:
        k = "x".join(map(str, gp.layout()))
        layouts[k] = layouts.get(k, 0) + 1
    line = {
        "metric": "walker proposals/s at matched final chi2",
        "value": proposals / elapsed,
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{len(jobs)} independent inversions in shared launches: N_omega in {{128,256,512,1024}} on "
                        "[0,20], N_tau in {32,64,128,256} on [0.02,3], walkers in {256,1024,4096}, 2-3 seeded "
                        "Lorentzians, noise log-uniform in [1e-6,1e-3] F, FP32 loop with FP64 resync every 50 "
                        "sweeps, T 1e3->1e-2 (x chi2_0) over 1000 sweeps, imprinted branching every 100",
            "n_jobs": len(jobs), "sweeps_timed": swept, "precision": "fp32 loop",
            "layouts_lanes_x_tau_per_lane": layouts,
        },
        "jobs_per_s": len(jobs) * swept / n_sweeps / elapsed,
        "quality": {
            "final_chi2_over_chi2_0_median_over_jobs": float(np.median(rel)),
            "final_chi2_over_chi2_0_max_over_jobs": float(rel.max()),
            "at_sweep": swept,
        },
        "roofline": {
            "kernel": "k_sweep_batched<float>",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": measured_traffic(args.workload),
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "avg_launch_ms": sweep_ms / launches,
            "launches": launches,
            "sweep_share_of_step": sweep_ms / (elapsed * 1e3),
        },
        "autotune_s": t_tune,
    }
    if plain is not None:
        line["plain_fp64_one_at_a_time"] = plain
        line["speedup_over_plain_fp64"] = {"proposals_per_s": line["value"] / plain["proposals_per_s"],
                                           "solves_per_s": line["jobs_per_s"] / plain["solves_per_s"]}
    if not args.no_cpu_baseline:
        # the oracle on the first four jobs, a walker sample of each, 400 sweeps
        tot_p, tot_t = 0, 0.0
        for wl in jobs[:4]:
            T = W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps)
            cb = cpu_baseline(wl, T, min(512, wl.n_walkers), 400)
            n_prop = min(512, wl.n_walkers) * wl.omega.size * 400
            tot_p += n_prop
            tot_t += n_prop / cb["value"]
        line["cpu_baseline"] = {"value": tot_p / tot_t, "unit": "proposals/s", "cores": cb["cores"],
                                "cpu_model": cb["cpu_model"], "kind": "oracle",
                                "sample": f"first 4 jobs, up to 512 walkers each (evenly strided), sweeps 0-399, "
                                          f"sweeps only: {tot_p} proposals in {tot_t:.2f} s"}
    return line


def served(args):
    print(json.dumps(served_line(args)), flush=True)


def served_line(args) -> dict:
    """Jobs of the batched workload's distribution (1000 sweeps each) arrive
    as a Poisson stream into the server; reports completed solves/s over the
    whole run and the submit-to-result latency percentiles, with sequential
    solo solves of the first jobs as the comparison."""
    import threading
    import torch
    from paper_1609_07936_amd import sail as S
    from paper_1609_07936_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    rng = np.random.default_rng(5)  # arrival seed
    n_jobs = max(1, int(rng.poisson(args.rate * args.duration)))
    arrivals = np.sort(rng.uniform(0.0, args.duration, n_jobs))
    jobs = W.batch_jobs(n_jobs, base_seed=20000)
    scheds = [S.Schedule(W.geometric_schedule(wl.t_hi, wl.t_lo, wl.n_sweeps), branch_every=wl.branch_every,
                         resync_every=wl.resync_every) for wl in jobs]
    # layouts of every shape tuned before the clock starts
    shapes = {}
    for wl in jobs:
        shapes.setdefault((wl.omega.size, wl.tau.size, wl.n_walkers), wl)
    for wl in shapes.values():
        S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1).autotune_layout(wl.n_walkers, S.SAIL_FP32)
    # the comparison: the first jobs solved one at a time on the plain FP64 path
    k = min(max(1, args.plain_jobs), n_jobs)
    plain = plain_fp64_solves(S, W, jobs[:k], scheds[:k])
    srv = S.Server(hbm_bytes=64 << 30, max_jobs=args.max_jobs)
    ids = [None] * n_jobs
    t_base = srv.clock()

    def submitter():
        for i, (wl, sc) in enumerate(zip(jobs, scheds)):
            dt = t_base + arrivals[i] - srv.clock()
            if dt > 0:
                time.sleep(dt)
            ids[i] = srv.submit(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1, wl.n_walkers, wl.seed, sc,
                                precision=S.SAIL_FP32)

    th = threading.Thread(target=submitter)
    th.start()
    res = []
    for i in range(n_jobs):
        while ids[i] is None:
            time.sleep(0.001)
        res.append(srv.wait(ids[i]))
        if i % 200 == 0:
            print(f"served {i + 1}/{n_jobs} at {srv.clock() - t_base:.1f} s", file=sys.stderr, flush=True)
    th.join()
    st = srv.stats()
    srv.close()
    ok = [r for r in res if r["status"] == 0]
    lat = np.array([r["t_done"] - r["t_submit"] for r in ok])
    wait = np.array([r["t_admit"] - r["t_submit"] for r in ok])
    # a sustainable load keeps latency flat over the window: compare the jobs
    # that arrived in its first and second halves
    sub = np.array([r["t_submit"] - t_base for r in ok])
    first, second = lat[sub < args.duration / 2], lat[sub >= args.duration / 2]
    span = max(r["t_done"] for r in ok) - t_base
    prop = sum(wl.n_walkers * wl.omega.size * wl.n_sweeps for wl, r in zip(jobs, res) if r["status"] == 0)
    flops = 8.0 * sum(wl.n_walkers * wl.omega.size * wl.tau.size * wl.n_sweeps for wl, r in zip(jobs, res)
                      if r["status"] == 0)
    rel = np.array([r["chi2_median"] / r["chi2_unit"] for r in ok])
    achieved = flops / (st["sweep_ms"] * 1e-3) / 1e12
    line = {
        "metric": "solves/s with p50/p99 latency at matched final chi2",
        "value": len(ok) / span,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(ok),
        "warmup": 0,
        "ms_per_step": span / max(1, len(ok)) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"Poisson arrivals at {args.rate:g} jobs/s for {args.duration:g} s of mixed-size "
                        "jobs (N_omega in {128..1024}, N_tau in {32..256}, walkers in {256,1024,4096}, 1000 "
                        "sweeps, FP32 loop, FP64 resync every 50, branching every 100) into one server "
                        f"(64 GiB arena, at most {args.max_jobs} in flight)",
            "offered_jobs": n_jobs, "rate": args.rate, "duration_s": args.duration,
        },
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max()), "queue_wait_p50": float(np.percentile(wait, 50)),
                      "queue_wait_p99": float(np.percentile(wait, 99)),
                      "p50_first_half_arrivals": float(np.percentile(first, 50)) if first.size else None,
                      "p50_second_half_arrivals": float(np.percentile(second, 50)) if second.size else None,
                      "p99_second_half_arrivals": float(np.percentile(second, 99)) if second.size else None},
        "sustained": bool(first.size and second.size and np.percentile(second, 50) < 1.5 * np.percentile(first, 50)
                          and len(ok) / span > 0.9 * args.rate),
        "proposals_per_s": prop / span,
        "plain_fp64_one_at_a_time": plain,
        "speedup_over_plain_fp64": {"solves_per_s": (len(ok) / span) / plain["solves_per_s"]},
        "failed": len(res) - len(ok),
        "quality": {"final_chi2_over_chi2_0_median_over_jobs": float(np.median(rel))},
        "roofline": {"kernel": "k_sweep_batched<float>", "bound": "alu", "achieved": achieved,
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": None, "avg_launch_ms": st["sweep_ms"] / max(1, st["sweep_launches"]),
                     "launches": st["sweep_launches"]},
        "server": st,
    }
    served_rel = {i: r["chi2_median"] / r["chi2_unit"] for i, r in enumerate(res[:k]) if r["status"] == 0}
    plain["median_final_chi2_ratio_served_over_plain"] = [float(served_rel[i] / plain["final_chi2_over_chi2_0_median"][i])
                                                          for i in served_rel]
    plain["matched_final_chi2"] = all(matched(served_rel[i], plain["final_chi2_over_chi2_0_median"][i])
                                      for i in served_rel)
    return line


def band(args):
    """The paper's model (Eq. lorentzian-band) with its protocol: self-cooling
    (20 boiling and 100 cooling blocks of 100 sweeps, then freeze-out),
    smoothing 0.01 and adaptive branching, 1500 walkers, 1000 bins; reports
    proposals/s, the skew of Sec. 5.3 and the recovered peak positions."""
    import torch
    from paper_1609_07936_amd import sail as S
    from paper_1609_07936_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = W.paper_band(args.band_noise, n_seq=args.n_seq, level=args.level, n_sweeps=args.band_sweeps)
    blocks = wl.n_sweeps // SWEEPS_PER_STEP
    steps = blocks  # the skew is a property of the whole anneal
    stream = torch.cuda.current_stream()
    sched = S.Schedule(np.ones(wl.n_sweeps), branch_every=SWEEPS_PER_STEP, resync_every=SWEEPS_PER_STEP,
                       smooth=0.01, adaptive=1, self_cool=1, boil_blocks=20, cool_blocks=args.band_cool)
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    # 1500 walkers fill few CUs, and the job has the device to itself: the smallest tile is a candidate
    gp.autotune_layout(wl.n_walkers, S.SAIL_FP64, stream=stream, alone=True)
    gp.init_walkers(wl.n_walkers, wl.seed, stream=stream)
    gp.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        gp.run(sched, s * SWEEPS_PER_STEP, SWEEPS_PER_STEP, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sweep_ms, launches = gp.sweep_timing(reset=True)
    proposals = wl.n_walkers * wl.omega.size * SWEEPS_PER_STEP * steps
    spec = gp.read_spectrum(stream=stream)
    chi2 = gp.read_chi2(stream=stream)
    left, right = wl.omega < 1.5, wl.omega >= 1.5
    flops = 8.0 * wl.tau.size * proposals
    achieved = flops / (sweep_ms * 1e-3) / 1e12
    line = {
        "metric": "walker proposals/s at matched final chi2",
        "value": proposals / elapsed,
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "paper's two-peak Lorentzian band: L(1, 1) + L(2, 1) clipped to [0.5, 2.5], 1000 bins on "
                        f"[0, 3.5], {wl.tau.size} tau from 0 step {wl.tau[1]:g}, {wl.n_walkers} walkers, "
                        f"{SWEEPS_PER_STEP * steps} sweeps, self-cooling (20 boil + {args.band_cool} cool blocks of 100 "
                        "sweeps), "
                        "smoothing 0.01, adaptive branching",
            "noise": args.band_noise, "level": args.level if args.band_noise == "iid" else None,
            "n_seq": args.n_seq if args.band_noise == "resampled" else None,
            "relative_sigma_tau0": None if wl.sigma is None else float(wl.sigma[0] / wl.F_true[0]),
            "layout_lanes_x_tau_per_lane": list(gp.layout()),
        },
        "quality": {
            "skew": W.band_skew(spec, wl.omega),
            "paper_skew_noiseless_1e-5_1e-4": [0.004, 0.017, 0.05],
            "peaks": [float(wl.omega[left][np.argmax(spec[left])]), float(wl.omega[right][np.argmax(spec[right])])],
            "final_chi2_over_chi2_0_median": float(np.median(chi2) / gp.chi2_unit),
            "at_sweep": SWEEPS_PER_STEP * steps,
        },
        "roofline": {"kernel": "k_sweep<double>", "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "avg_launch_ms": sweep_ms / launches, "launches": launches,
                     "sweep_share_of_step": sweep_ms / (elapsed * 1e3)},
    }
    print(json.dumps(line), flush=True)


def extras(args) -> dict:
    """The batched and served workloads measured in the same run as the
    default line, summarised: each against the same jobs solved one at a time
    on the plain FP64 path."""
    import copy
    a = copy.copy(args)
    a.steps, a.warmup, a.no_cpu_baseline = 10 ** 6, 1, True
    b = batched_line(a)
    a.rate, a.duration = args.extras_rate, args.extras_duration
    v = served_line(a)
    keep = ("metric", "value", "unit", "ms_per_step", "jobs_per_s", "roofline", "plain_fp64_one_at_a_time",
            "speedup_over_plain_fp64", "latency_s", "sustained", "proposals_per_s", "failed", "quality")
    out = {"batched": {k: b[k] for k in keep if k in b}, "served": {k: v[k] for k in keep if k in v}}
    out["batched"]["workload"] = b["config"]["workload"]
    out["served"]["workload"] = v["config"]["workload"]
    out["served"]["roofline"] = {k: v["roofline"][k] for k in ("achieved", "frac", "avg_launch_ms")}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the anneal runs on one device)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return batched(args)
    if args.workload == "served":
        return served(args)
    if args.workload == "band":
        return band(args)
    import torch
    from paper_1609_07936_amd import sail as S
    from paper_1609_07936_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    fp32 = args.workload == "fp32"
    wl = W.large_512x128_fp32() if fp32 else W.large_512x128()
    precision = S.SAIL_FP32 if fp32 else S.SAIL_FP64
    n_sweeps_total = wl.n_sweeps
    T = W.geometric_schedule(wl.t_hi, wl.t_lo, n_sweeps_total)
    steps, warm = args.steps, args.warmup
    if steps * SWEEPS_PER_STEP > n_sweeps_total:
        raise SystemExit("steps exceed the schedule")
    stream = torch.cuda.current_stream()
    gp = S.Problem(wl.omega, wl.tau, wl.Ft, wl.sigma, wl.m0, wl.m1)
    boil, cool = (int(x) for x in args.self_cool.split(",")) if args.self_cool else (0, 1)
    sched = S.Schedule(T, branch_every=SWEEPS_PER_STEP, resync_every=wl.resync_every, smooth=args.smooth,
                       adaptive=int(args.adaptive), self_cool=int(bool(args.self_cool)), boil_blocks=boil,
                       cool_blocks=cool)
    if args.tpl:
        gp.set_tau_per_lane(args.tpl)
    gp.init_walkers(wl.n_walkers, wl.seed, precision=precision, stream=stream)
    for s in range(warm):
        gp.run(sched, s * SWEEPS_PER_STEP, SWEEPS_PER_STEP, stream=stream)
    torch.cuda.synchronize()
    # the timed anneal starts from fresh walkers at sweep 0
    gp.init_walkers(wl.n_walkers, wl.seed, precision=precision, stream=stream)
    gp.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        gp.run(sched, s * SWEEPS_PER_STEP, SWEEPS_PER_STEP, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sweep_ms, launches = gp.sweep_timing(reset=True)
    gp.set_timing(False)
    elapsed = t1 - t0
    proposals = wl.n_walkers * wl.omega.size * SWEEPS_PER_STEP * steps
    value = proposals / elapsed
    chi2 = gp.read_chi2(stream=stream)
    total_steps = n_sweeps_total // SWEEPS_PER_STEP
    quality = {
        "timed_region_chi2_over_chi2_0_median": float(np.median(chi2) / gp.chi2_unit),
        "timed_region_chi2_over_chi2_0_min": float(chi2.min() / gp.chi2_unit),
        "timed_region_ends_at_sweep": SWEEPS_PER_STEP * steps,
    }
    chi2_final = chi2 if steps == total_steps else None
    if chi2_final is None and not args.no_finish:
        # the rest of the same anneal, untimed, so that the final residues are measured
        t2 = time.perf_counter()
        for s in range(steps, total_steps):
            gp.run(sched, s * SWEEPS_PER_STEP, SWEEPS_PER_STEP, stream=stream)
        chi2_final = gp.read_chi2(stream=stream)
        quality["untimed_rest_s"] = time.perf_counter() - t2
    if chi2_final is not None:
        quality.update({
            "final_chi2_over_chi2_0_median": float(np.median(chi2_final) / gp.chi2_unit),
            "final_chi2_over_chi2_0_min": float(chi2_final.min() / gp.chi2_unit),
            "final_at_sweep": n_sweeps_total,
        })
    # roofline of the sweep kernel: 8 N_tau algorithmic flops per proposal
    flops_per_launch = 8.0 * wl.tau.size * wl.n_walkers * wl.omega.size * (SWEEPS_PER_STEP * steps / launches)
    avg_ms = sweep_ms / launches
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    peak = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
    line = {
        "metric": "walker proposals/s at matched final chi2",
        "value": value,
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": ("FP32-loop variant (FP64 resync + renormalisation every 50 sweeps) of the " if fp32 else
                         "production FP64 anneal: ") +
                        "512 omega bins on [0,20], 128 uniform tau on [0.02,3], "
                        "16384 walkers, T 1e3->1e-2 (x chi2_0) geometric over 20000 sweeps, blocks of 100 sweeps "
                        "with resync + imprinted branching (fraction 1/4, t = 0.1); seeded two-Lorentzian target, "
                        "noise 1e-5 F",
            "n_omega": int(wl.omega.size), "n_tau": int(wl.tau.size), "n_walkers": int(wl.n_walkers),
            "sweeps_timed": SWEEPS_PER_STEP * steps, "precision": "fp32 loop" if fp32 else "fp64",
            "smooth": args.smooth, "adaptive_branching": bool(args.adaptive),
            "self_cooling_boil_cool_blocks": args.self_cool or None,
            "layout_lanes_x_tau_per_lane": list(gp.layout()),
        },
        "quality": quality,
        "roofline": {
            "kernel": "k_sweep<float>" if fp32 else "k_sweep<double>",
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": measured_traffic(args.workload),
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "lds": measured_lds(args.workload, avg_ms),
            "avg_launch_ms": avg_ms,
            "launches": launches,
            "sweep_share_of_step": sweep_ms / (elapsed * 1e3),
        },
    }
    if fp32 and chi2_final is not None and not args.self_cool:
        line["vs_fp64"] = fp64_comparison(S, W, wl, T, gp, chi2_final, value, stream, args.smooth,
                                          int(args.adaptive))
    if not fp32 and chi2_final is not None and not args.no_precision_match:
        line["precision_match"] = fp32_match(S, W, gp, chi2_final, sched, stream)
    if not fp32 and not args.no_extras:
        line["extras"] = extras(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, T, args.cpu_sample_walkers, args.cpu_sample_sweeps,
                                            one_thread_walkers=max(1, args.cpu_sample_walkers // 16))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
