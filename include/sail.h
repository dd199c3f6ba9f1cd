/*
 * sail.h -- C ABI of the MI355X (gfx950) implementation of the simulated
 * annealing inverse Laplace transform of Lutsyshyn & Astrakharchik
 * ("SAIL", arXiv:1609.07936).
 *
 * The library anneals a population of walkers, each a piecewise-constant
 * spectrum a_j >= 0 on N_omega uniform bins (Sec. 2.1, Eq. spectral-model),
 * against data F(tau_i) with errors sigma_i.  Every proposal is the
 * sum-rule preserving two-bin move of Sec. 2.2 (Eqs. update-scheme-p/s/j,
 * update-delta-p/s); the reconstruction F(tau) is updated incrementally
 * (Sec. 2.2, F' = r F + dp K_p + ds K_s) and the residue change is reduced
 * over all tau points and accepted by the Metropolis rule at the current
 * temperature (Eq. probability-density).  After every block of sweeps the
 * walkers are branched with imprinting (Sec. 2.5).
 *
 * Conventions for every entry point:
 *  - Plain C types only.  Host pointers are marked "host", device pointers
 *    "device".  Input arrays are copied; the caller keeps ownership.
 *  - Output arrays are caller-allocated.
 *  - Every call returns a sail_status; nothing throws or aborts across the
 *    ABI.  On an error the call changes no state (one exception:
 *    sail_walkers_init, see there), and sail_last_error() returns a message
 *    for the calling thread.
 *  - A problem is used from one host thread at a time.  Work is enqueued on
 *    the HIP stream passed as `stream` (NULL means the null stream); calls
 *    that return host data synchronise that stream.
 */
#ifndef SAIL_H
#define SAIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sail_problem *sail_problem_t;

typedef enum {
    SAIL_OK = 0,
    SAIL_EINVAL = 1,      /* an argument is out of range or inconsistent */
    SAIL_EINFEASIBLE = 2, /* the two sum rules admit no non-negative spectrum */
    SAIL_ENOMEM = 3,      /* device or host allocation failed */
    SAIL_EDEVICE = 4,     /* a HIP runtime call failed */
    SAIL_ENUMERIC = 5,    /* a non-finite residue was found */
    SAIL_ESTATE = 6,      /* call out of order (e.g. run before init) */
    SAIL_ETIMEOUT = 7,    /* a wait ended before its job did */
    SAIL_ECANCELLED = 8   /* the server shut down before the job finished */
} sail_status;

typedef enum {
    /* K(omega_j, tau) = d_omega e^{-omega_j tau} / (2 pi): each bin sampled
     * at its centre. */
    SAIL_K_POINT = 0,
    /* K(omega_j, tau) = (1/2 pi) int over bin j of e^{-omega tau} d omega, the
     * exact bin integral of Eq. (correlation-model). */
    SAIL_K_BIN_EXACT = 1
} sail_kernel_mode;

typedef enum {
    SAIL_FP64 = 0, /* residual loop and residue change in FP64 */
    SAIL_FP32 = 1  /* residual loop in FP32, resync and final residue in FP64 */
} sail_precision;

/* Annealing schedule; defaults in brackets (those of the first fields from Sec. 3). */
typedef struct {
    const double *T;        /* host, n_T temperatures; sweep k runs at T[k] */
    int n_T;
    int branch_every;       /* sweeps per block; a branching event follows every block [100] */
    int resync_every;       /* exact recomputation of F and chi^2 every this many sweeps; divides branch_every */
    double branch_fraction; /* share of walkers given multiplier zero per event [0.25] */
    double imprint_t;       /* imprint strength t, a <- t a_donor + (1 - t) a [0.1] */
    double eps0;            /* width of 1 - r: r = 1 - y eps0 (2u - 1), 0 < eps0 < 1 [0.1] */
    double amp_p;           /* p of Eq. (amplitude-acceptance-adjustment) [1] */
    int amp_m;              /* m of the same equation, integer >= 0 [2] */
    double amp_avg;         /* weight of the newest sweep in the running acceptance rate, (0, 1] [0.1] */
    int walk_len;           /* steps of the index-selection walk of Sec. 2.3, 0..64 (0: uniform) [0] */
    int t_units;            /* 0: T in units of the starting residue (Sec. 3); 1: absolute */
    double smooth;          /* amplitude s of the three-point smoothing stencil of Sec. 2.6, [0, 0.5]
                               (0: off) [0]: after every branching event each walker's spectrum is
                               smoothed (a_j <- s a_{j-1} + (1 - 2s) a_j + s a_{j+1}, ends
                               (1 - s) a_end + s a_next), both sums renormalised, F and chi^2
                               recomputed */
    int adaptive;           /* 1: adaptive branching (Sec. 2.5, last paragraph) [0]: each event uses
                               branch_fraction and imprint_t scaled by the population mean of the
                               walkers' running acceptance rates (which start at 1) */
    int self_cool;          /* 1: self-cooling (Sec. 2.4) [0]; T then only sets the length (its values
                               must still be positive and finite),
                               and block b (branch_every sweeps) runs at a temperature taken from the
                               residues at its start: the mean for b < boil_blocks, then a linear ramp
                               from the mean to the minimum over cool_blocks blocks, then
                               min / (1 + j) in freeze block j = 1, 2, ...; a call starts at a block
                               boundary or inside the block the previous call started */
    int boil_blocks;        /* >= 0 [0] */
    int cool_blocks;        /* >= 1 [1] */
} sail_schedule;

/* Fills *s with the defaults above and T = NULL, n_T = 0. */
void sail_schedule_defaults(sail_schedule *s);

/* Creates a problem (Sec. 2.1).
 *   omega  host, n_omega >= 3 bin centres, uniform spacing (1e-12 relative)
 *   tau    host, n_tau >= 1 times >= 0, uniform spacing (1e-12 relative)
 *   F      host, n_tau data values
 *   sigma  host, n_tau errors > 0, or NULL for the paper's unweighted residue
 *   m0, m1 zeroth and first moment of the spectrum, int S and int omega S
 *          (Sec. 2.2: A = m0 / d_omega, B = m1 / d_omega)
 *   kernel_mode  a sail_kernel_mode
 *   device HIP device ordinal the problem lives on
 * SAIL_EINFEASIBLE if m1 / m0 is not strictly inside (omega_0, omega_{n-1}).
 * Limits (SAIL_EINVAL beyond them): n_tau <= 1024 (64 lanes of 16 tau
 * points per walker); n_omega as far as one workgroup's LDS holds the
 * resync's staged spectra (n_omega <= 2556 on gfx950). */
sail_status sail_problem_create(const double *omega, int n_omega, const double *tau, int n_tau,
                                const double *F, const double *sigma, double m0, double m1,
                                int kernel_mode, int device, sail_problem_t *out);

/* Releases all device and host memory of the problem.  NULL is ignored. */
void sail_problem_destroy(sail_problem_t p);

/* Allocates n_walkers walkers and sets each to the maximum-entropy spectrum
 * a_j ~ e^{-lambda omega_j} meeting both sum rules, computes F = K a and the
 * starting residue chi^2_0 (the unit of temperature, Sec. 3).  `seed` keys
 * the Philox4x32-10 stream of every random draw.  Resets the sweep and
 * event logs.  n_walkers >= 2, and n_walkers * n_omega doubles of spectra
 * below 2 GiB; sail_run_schedule takes at most 16384 walkers (the
 * branching solve's reach).  The previous walkers (and their logs, trace
 * window aside) are released first, so that the new population can use
 * their memory: after a failed call the problem holds no walkers and the
 * calls that need them return SAIL_ESTATE until an initialisation succeeds. */
sail_status sail_walkers_init(sail_problem_t p, int n_walkers, uint64_t seed, int precision, void *stream);

/* Runs global sweeps [first_sweep, first_sweep + n_sweeps) of `sched`.
 * A sweep is n_omega proposals per walker.  After sweep k, if (k + 1) is a
 * multiple of resync_every every walker is renormalised to both sum rules and
 * its F and chi^2 recomputed; if (k + 1) is a multiple of branch_every the
 * branching event (k + 1) / branch_every - 1 follows (Sec. 2.5; with 256
 * walkers or more its Delta search runs over many workgroups, with the
 * same result).  Stages may be run in several calls; the random stream
 * depends only on the global sweep, proposal and walker indices. */
sail_status sail_run_schedule(sail_problem_t p, const sail_schedule *sched, int first_sweep, int n_sweeps,
                              void *stream);

/* Starting residue chi^2_0 (absolute units), or NaN before init. */
double sail_chi2_unit(sail_problem_t p);

/* Ensemble-mean spectrum, out: host, n_omega doubles (Eq. residue-average
 * estimated over the walkers). */
sail_status sail_read_spectrum(sail_problem_t p, double *out, void *stream);

/* Watchdog (failure detection) for sail_run_schedule.  With drift_bound > 0
 * every resync inside a call checks every walker: a residue that is not
 * finite, or (at the plain renormalising resync) a relative drift of either
 * sum rule, |sum a - A| / A or |sum omega a - B| / B (Sec. 2.2: both are
 * invariants of every move), above drift_bound before the renormalisation.
 * The walker state at the call's start and after every clean resync
 * boundary (after its branching event, if any) is kept as a snapshot on the
 * device; when a check trips, the call still finishes its launches, then
 * restores the last snapshot and returns SAIL_ENUMERIC: the walkers are as
 * they were at that sweep (sail_watchdog_report gives it), and a run may be
 * resumed from there.  drift_bound = 0 switches the watchdog off.  Needs
 * walkers (SAIL_ESTATE before sail_walkers_init; re-initialising switches it
 * off); the snapshot doubles the walker state's device memory.  Batches and
 * served jobs do not run it. */
sail_status sail_set_watchdog(sail_problem_t p, double drift_bound);
/* Of the last sail_run_schedule call: the sweep after which a check tripped
 * and the sweep the walkers were restored to, both -1 if none tripped. */
sail_status sail_watchdog_report(sail_problem_t p, int *tripped_after_sweep, int *restored_to_sweep);

/* Per-block log (the temperature, residue and acceptance rate the paper's
 * program reports after each block, Sec. 4).  With capacity > 0,
 * sail_run_schedule appends one record at every resync boundary, after the
 * boundary's branching event if there is one, to a device ring of the last
 * `capacity` records; one workgroup reduces the population in a fixed order,
 * so records are deterministic.  Statistics over all walkers: */
typedef struct {
    int32_t sweep;     /* sweeps completed when the block ended */
    int32_t event;     /* the boundary's branching event (index in the event log), or -1 */
    double T;          /* absolute temperature of the block's last sweep */
    double chi2_min;   /* residues after the resync and branching */
    double chi2_mean;
    double chi2_median; /* numpy's median: the middle residue, or the mean of the two */
    double chi2_max;
    double rate_mean;  /* running acceptance rate (Sec. 2.7), mean over walkers */
    double drift_max;  /* largest relative sum-rule drift, max(|sum a - A| / A,
                          |sum omega a - B| / |B|), found by the boundary's
                          renormalising resync before it renormalised */
} sail_block_record;
/* capacity = 0 switches the log off.  Needs walkers (SAIL_ESTATE otherwise);
 * every call, and sail_walkers_init, empties the log; records of blocks that
 * a watchdog rollback undoes stay in it (their sweep numbers repeat when the
 * run resumes).  Device memory:
 * capacity records of 64 bytes plus one double per walker.  A problem run
 * in a batch keeps its log too (the same records as alone); served jobs keep
 * none. */
sail_status sail_set_block_log(sail_problem_t p, int capacity);
/* Copies the newest min(max_records, records held) records, oldest first,
 * into out (host, caller-allocated) on `stream` and synchronises it;
 * *n_records receives how many, *n_total how many were appended since the
 * log was switched on (either may be NULL).  SAIL_ESTATE when the log is
 * off. */
sail_status sail_read_block_log(sail_problem_t p, sail_block_record *out, int max_records, int *n_records,
                                int64_t *n_total, void *stream);

/* Current residue chi^2 (Eq. residue, weighted by 1 / sigma_i^2 when sigma
 * was given) of every walker, exact as of the last resync plus the summed
 * changes of the accepted moves since; out: host, n_walkers doubles. */
sail_status sail_read_chi2(sail_problem_t p, double *out, void *stream);

/* Histogram of log10 chi^2 over the walkers, over [lo, hi) in n_bins bins,
 * 1 <= n_bins <= 4096 (values outside are clamped into the end bins).  A
 * library output, not a quantity of the paper: it summarises the spread of
 * the population's residues between its mean and minimum, which drive the
 * self-cooling prescription of Sec. 2.4 (residues in the unit of Sec. 3).
 * If lo or hi is NaN the ensemble minimum / maximum is used.
 * counts: host, n_bins uint64.  Allocates and frees a device buffer for the
 * counts on every call. */
sail_status sail_read_chi2_hist(sail_problem_t p, int n_bins, double lo, double hi, uint64_t *counts,
                                void *stream);

/* The same histogram for callers that cannot allocate device memory (code
 * recorded under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): identical arguments and results, but the call makes no
 * hipMalloc / hipFree or other allocating call.  Its scratch (the range and
 * the counts) is a device-resident array inside the library, one per device,
 * held until the process ends; its first call on a device looks up that
 * device's copy.  n_bins above 4096 (the array's size) is SAIL_EINVAL.
 * counts: host or device memory, n_bins uint64, written by a copy on
 * `stream`, which the call synchronises.  Every call on one device shares
 * that device's array: calls that overlap on one device (other threads or
 * streams) race and must be serialised by the caller. */
sail_status sail_read_chi2_hist_noalloc(sail_problem_t p, int n_bins, double lo, double hi, uint64_t *counts,
                                        void *stream);

/* Walker state, every pointer host and optional (NULL skips it):
 *   a     [n_walkers][n_omega] spectra a_j (scale folded in)
 *   F     [n_walkers][n_tau] reconstructions F(tau_i)
 *   rate  [n_walkers] running acceptance rates */
sail_status sail_read_state(sail_problem_t p, double *a, double *F, double *rate, void *stream);

/* Branching log of events [0, n_events): Delta, P_r, zero count, status
 * (0 done, 1 skipped: target unreachable, 2 skipped: threshold tie), and
 * optionally the multipliers m, [n_events][n_walkers] (requires
 * sail_set_event_log(p, 1) before the events ran).  Host pointers, any may
 * be NULL. */
sail_status sail_read_events(sail_problem_t p, int n_events, double *delta, double *pr, int32_t *z,
                             int32_t *status, int32_t *m);
/* Keeps the multipliers of every later event (keep_multipliers = 1; each
 * such call starts an empty multiplier log) or stops keeping them (0).
 * Needs initialised walkers; a failed call (SAIL_ENOMEM) changes nothing. */
sail_status sail_set_event_log(sail_problem_t p, int keep_multipliers);

/* Margins of the branching solves of events [0, n_events) (Sec. 2.5), host
 * pointers, either may be NULL:
 *   gap      the distance between the n-th and (n+1)-th smallest thresholds
 *            theta_{l,k} = chi^2_l + ln(k - xi_l) / Delta at the final Delta
 *            (P_r is their midpoint), relative to the larger of their
 *            magnitudes and 1 / Delta; small by construction, since the
 *            search for Delta ends just above the crossing of two thresholds
 *            that moves the zero count
 *   bracket  the relative width (hi - lo) / hi of the final bracket of that
 *            search; the crossing lies inside it, below Delta
 * Skipped events hold +infinity. */
sail_status sail_read_event_margins(sail_problem_t p, int n_events, double *gap, double *bracket);

/* Per-proposal trace of global sweeps [k0, k1) for every walker into device
 * buffers laid out [walker][sweep - k0][proposal]:
 *   dchi2  device, the residue change of the proposal (computed for every
 *          proposal, also rejected ones)
 *   flags  device, bit 0 accepted, bit 1 admissible (p != s and a' >= 0)
 * k0 == k1 switches tracing off.  The buffers must stay valid while sweeps
 * in the window run.  Tracing selects a slower kernel variant. */
sail_status sail_set_trace(sail_problem_t p, int k0, int k1, double *dchi2, uint8_t *flags);

/* Timing of the sweep kernel with HIP events on the launch stream: when
 * enabled, every sweep launch is bracketed by events; sail_sweep_timing
 * synchronises and returns the summed kernel time and launch count since the
 * last reset. */
sail_status sail_set_timing(sail_problem_t p, int enable);
sail_status sail_sweep_timing(sail_problem_t p, double *total_ms, int64_t *launches, int reset);

/* Checkpoint of the walker population (spectra, reconstructions, scales,
 * residues, acceptance rates, seed and residue unit); with the counter-based
 * random stream, export -> import -> continue is bit-identical to an
 * uninterrupted run.  Export: buf host; with buf == NULL only *bytes is set
 * to the size needed; otherwise *bytes is the capacity of buf on entry and
 * the size written on return.  Import: buf host, bytes its size; the problem
 * must already hold walkers of the same count, layout and precision
 * (sail_walkers_init). */
sail_status sail_state_export(sail_problem_t p, void *buf, size_t *bytes, void *stream);
sail_status sail_state_import(sail_problem_t p, const void *buf, size_t bytes, void *stream);

/* Batches: many independent problems annealed together on one device
 * (Sec. 2.5 and 3 per problem; the batch is a throughput device of this
 * library, not of the paper).  The batch refers to the problems; it does not
 * own them, and they must outlive it.  All problems live on one device and
 * each appears once.
 *
 * sail_batch_run runs, for every problem i, global sweeps
 * [first_sweep[i], first_sweep[i] + n_sweeps[i]) of *scheds[i] (host arrays of
 * n_problems entries), with exactly the semantics and the random stream of
 * sail_run_schedule on that problem alone: the results are bit-identical.
 * The problems advance in rounds, each taking every unfinished problem to
 * its next resync boundary in one shared sweep launch (per precision and
 * lane layout), followed by shared launches of the resyncs, the branching
 * solves and the imprints that fall due.  Problems may sit at different
 * sweeps and have different sizes, walker counts, precisions and schedules.
 * Traced sweeps (sail_set_trace) are refused.  Validation happens before any
 * work is enqueued. */
typedef struct sail_batch *sail_batch_t;
sail_status sail_batch_create(const sail_problem_t *problems, int n_problems, sail_batch_t *out);
void sail_batch_destroy(sail_batch_t b);
sail_status sail_batch_run(sail_batch_t b, const sail_schedule *const *scheds, const int *first_sweep,
                           const int *n_sweeps, void *stream);
/* Timing of the shared sweep launches, as sail_set_timing / sail_sweep_timing. */
sail_status sail_batch_set_timing(sail_batch_t b, int enable);
sail_status sail_batch_sweep_timing(sail_batch_t b, double *total_ms, int64_t *launches, int reset);

/* Served anneals: a server owns one device, a device arena of hbm_bytes and
 * a host thread.  Submitted jobs queue in arrival order; the head job is
 * admitted when at most max_jobs - 1 jobs are in flight and its footprint
 * (its tables, walker state, schedule and outputs) fits in the free part of
 * the arena, so the device memory of all in-flight jobs never exceeds
 * hbm_bytes and no device allocation happens per job.  Admitted jobs keep all
 * state on the device and advance together in the rounds of sail_batch_run:
 * every round one shared sweep launch takes each in-flight job, whatever its
 * stage, to its next resync boundary, and jobs join or leave between rounds
 * (continuous batching).  A job runs its whole schedule (sweeps [0, n_T)) from
 * sail_walkers_init, with the semantics and random stream of
 * sail_run_schedule: its outputs are bit-identical to the same job run alone.
 * Times are seconds on the server's monotonic clock (sail_server_clock). */
typedef struct sail_server *sail_server_t;

typedef struct {
    int device;
    size_t hbm_bytes; /* device arena; admission budget of all in-flight jobs */
    int max_jobs;     /* in-flight jobs at most */
} sail_server_config;

typedef struct {
    /* the problem, as sail_problem_create (host arrays, copied at submit) */
    const double *omega; int n_omega;
    const double *tau; int n_tau;
    const double *F; const double *sigma;
    double m0, m1;
    int kernel_mode;
    /* the walkers, as sail_walkers_init */
    int n_walkers;
    uint64_t seed;
    int precision;
    int tau_per_lane;      /* as sail_set_tau_per_lane; -1: sail_autotune_layout */
    sail_schedule sched;   /* T copied at submit; all n_T sweeps run */
} sail_job;

typedef struct {
    int status;                       /* sail_status of the job */
    double t_submit, t_admit, t_done; /* server clock */
    double chi2_unit;                 /* starting residue chi^2_0 */
    double chi2_min, chi2_median;     /* final residues over the walkers */
    int n_omega, n_walkers;
} sail_job_result;

typedef struct {
    int64_t submitted, admitted, completed, failed;
    int queued, in_flight;
    size_t arena_bytes, arena_used, arena_peak;
    int64_t rounds;
    double sweep_ms; /* summed duration of the shared sweep launches */
    int64_t sweep_launches;
    int64_t cancelled; /* jobs ended with SAIL_ECANCELLED (sail_server_cancel or shutdown) */
} sail_server_stats;

/* Job states reported by sail_server_poll. */
enum { SAIL_JOB_QUEUED = 0, SAIL_JOB_RUNNING = 1, SAIL_JOB_DONE = 2 };

/* Starts the server thread.  SAIL_ENOMEM if the arena cannot be allocated. */
sail_status sail_server_create(const sail_server_config *cfg, sail_server_t *out);
/* Queues a job (thread-safe); inputs are validated as by sail_problem_create /
 * sail_run_schedule where that needs no device (the rest is reported in the
 * job's result).  SAIL_EINVAL if the job could never fit the arena. */
sail_status sail_server_submit(sail_server_t s, const sail_job *job, int64_t *id);
/* Waits up to timeout_s seconds (< 0: no limit) for job `id`; on SAIL_OK fills
 * *res and, if mean_spectrum (host, n_omega doubles) is not NULL, the
 * ensemble-mean spectrum, and forgets the job.  SAIL_ETIMEOUT leaves it. */
sail_status sail_server_wait(sail_server_t s, int64_t id, double timeout_s, sail_job_result *res,
                             double *mean_spectrum);
/* State of job `id` without waiting (thread-safe): SAIL_JOB_QUEUED,
 * SAIL_JOB_RUNNING (admitted: in flight, or its outputs being read back) or
 * SAIL_JOB_DONE (sail_server_wait returns at once).  SAIL_EINVAL for an id
 * that is unknown or already waited for. */
sail_status sail_server_poll(sail_server_t s, int64_t id, int *state);
/* Cancels job `id` (thread-safe).  A queued job leaves the queue at once; a
 * running job leaves the shared rounds at the next round boundary and its
 * arena block returns once the device has finished the work already
 * enqueued for it; either way its result has status SAIL_ECANCELLED (collect
 * it with sail_server_wait).  SAIL_ESTATE if the job has already finished
 * its anneal (its result stands), SAIL_EINVAL for an unknown id. */
sail_status sail_server_cancel(sail_server_t s, int64_t id);
sail_status sail_server_get_stats(sail_server_t s, sail_server_stats *out);
double sail_server_clock(sail_server_t s);
/* Arena bytes a job takes while in flight (0 for a malformed job or schedule). */
size_t sail_job_footprint_bytes(const sail_job *job);
/* Stops the thread: queued and in-flight jobs end with SAIL_ECANCELLED (after
 * the device has finished their work), then frees everything. */
void sail_server_destroy(sail_server_t s);

/* Upper bound of the device bytes a problem of this size holds at this
 * precision (tables plus walker state, any lane layout), excluding the
 * temperature schedule (8 bytes per sweep) and event logs beyond 64 events. */
size_t sail_footprint_bytes(int n_omega, int n_tau, int n_walkers, int precision);

/* Lanes per walker and tau points per lane the sweep kernel uses. */
sail_status sail_layout(sail_problem_t p, int *lanes_per_walker, int *tau_per_lane);

/* Requests tau points per lane for the next sail_walkers_init: 4, 8 or 16
 * for FP64, 8, 16 or 32 for FP32, 0 for the library's choice (16).  A
 * request the precision does not take falls back to the choice.  The walkers
 * per wavefront follow as 64 / next_pow2(ceil(n_tau / tau_per_lane)); the
 * smaller tiles give each walker more lanes, which pays when too few walkers
 * fill the device.  The layout changes only the summation order of the
 * residue change.  Any other value: SAIL_EINVAL. */
sail_status sail_set_tau_per_lane(sail_problem_t p, int tau_per_lane);

/* Chooses the tau points per lane for this problem at n_walkers walkers and
 * `precision` by timing a few sweeps of each candidate layout on `stream`
 * (the two larger tiles of the precision: 8 and 16 for FP64, 16 and 32 for
 * FP32, the right candidates when the job will share the device with
 * others, as in a batch or the served loop), and requests it as
 * sail_set_tau_per_lane does (*tau_per_lane receives it, may be NULL).  The served loop tunes each new shape after the rounds
 * already enqueued have drained, so the candidates run on an otherwise idle
 * device.  Results are cached per (device architecture,
 * n_omega, n_tau, n_walkers, precision) for the life of the process, and
 * across processes when the environment variable SAIL_TUNE_CACHE names a
 * file (read at the first lookup; each new choice is appended as one text
 * line).  Leaves the problem without walkers: call it before
 * sail_walkers_init. */
sail_status sail_autotune_layout(sail_problem_t p, int n_walkers, int precision, int *tau_per_lane, void *stream);

/* As sail_autotune_layout, for a problem that will have the device to
 * itself: the smallest tile (4 tau points per lane for FP64, 8 for FP32) is
 * a candidate too.  More lanes per walker shorten each proposal's serial
 * chain for more total work, which wins when the walkers alone leave the
 * device underfilled and loses once other jobs fill it.  Its choices are
 * cached apart from sail_autotune_layout's (a SAIL_TUNE_CACHE line tagged
 * sail-tune-alone-v1). */
sail_status sail_autotune_layout_alone(sail_problem_t p, int n_walkers, int precision, int *tau_per_lane,
                                       void *stream);

/* Device memory from the caller's allocator (for instance a framework's
 * caching allocator, so the library's buffers count against its pool).
 * alloc(bytes, device, user) returns `bytes` of device memory on `device`
 * (the current HIP device of the calling thread), aligned to 256 bytes, or
 * NULL when it cannot (the library call then fails with SAIL_ENOMEM).
 * release(ptr, bytes, device, user) takes back a block that alloc returned,
 * with the same bytes and device; the library has synchronised that device
 * first, so no kernel still uses the block.  Both are called from the host
 * thread that makes the library call, or from a server's loop thread, and
 * must be safe to call from any thread.  The hook is process-wide and
 * serves every later device allocation of problems, batches, staging
 * buffers and server arenas; pinned host buffers and the fixed scratch
 * array stay with HIP.  Blocks are returned to the allocator that made
 * them, also after the hook is changed or cleared; the caller keeps the
 * functions and `user` valid until then.  Both NULL restores hipMalloc and
 * hipFree; exactly one NULL is SAIL_EINVAL. */
typedef void *(*sail_alloc_fn)(size_t bytes, int device, void *user);
typedef void (*sail_free_fn)(void *ptr, size_t bytes, int device, void *user);
sail_status sail_set_allocator(sail_alloc_fn alloc, sail_free_fn release, void *user);

const char *sail_status_string(int status);
const char *sail_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SAIL_H */
