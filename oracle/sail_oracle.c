/*
 * sail_oracle.c -- plain FP64 CPU oracle for the simulated-annealing inverse
 * Laplace transform of Lutsyshyn & Astrakharchik (SAIL, arXiv:1609.07936).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  This file is the slow, obviously
 * correct definition the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header, table or constant generator with the GPU library; the only
 * thing both sides have in common is the published definition of the
 * Philox4x32-10 counter-based generator, which each implements on its own.
 *
 * Every function cites the passage of the paper it follows.  Readings of
 * points the paper leaves open are marked "Reading:".  Build with
 * -O2 -ffp-contract=off so every a*b+c is two roundings, as written.
 *
 * Notation: omega_j are bin centres (the paper's omega_j + d_omega/2),
 * d_omega is uniform, K[j*n_tau+i] is the kernel table, w_i = 1/sigma_i^2,
 * A = sum_j a_j and B = sum_j a_j omega_j are the two conserved sums.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the */
/* round multipliers 0xD2511F53 / 0xCD9E8D57, key schedule bumped by the     */
/* Weyl constants 0x9E3779B9 / 0xBB67AE85 between rounds.                    */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Reading (RNG is unstated in the paper): a 32-bit word x maps to the open
 * unit interval as (x + 1/2) 2^-32, and to an index in [0, n) by the high
 * half of the 64-bit product x*n. */
static double u01(uint32_t x) { return ((double)x + 0.5) * 2.3283064365386962890625e-10; }
static int index_of(uint32_t x, int n) { return (int)(((uint64_t)x * (uint64_t)n) >> 32); }

/* Stream tags in the fourth counter word. */
#define OR_STREAM_PROPOSAL 0u
#define OR_STREAM_BRANCH 0x42524E43u

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Kernel table.  Sec. 2.1, Eq. (correlation-model): the transform of a     */
/* rectangle of height a_j on bin j is (a_j/2pi) int e^{-omega tau} d omega. */
/*   mode 0 (POINT): bin sampled at its centre, K = d_omega e^{-omega tau}/2pi */
/*   mode 1 (BIN_EXACT): the bin integral itself,                          */
/*        K = (e^{-lo tau} - e^{-hi tau}) / (2 pi tau),  K = d_omega/2pi at tau=0 */
/* ------------------------------------------------------------------------ */
int or_kernel_table(int mode, const double *omega, int n_omega, const double *tau, int n_tau, double *K)
{
    if (n_omega < 2 || n_tau < 1) return 1;
    double dw = omega[1] - omega[0];
    for (int j = 0; j < n_omega; ++j) {
        for (int i = 0; i < n_tau; ++i) {
            double t = tau[i], v;
            if (mode == 0) {
                v = dw / OR_TWO_PI * exp(-omega[j] * t);
            } else {
                double lo = omega[j] - 0.5 * dw, hi = omega[j] + 0.5 * dw;
                if (t == 0.0) v = dw / OR_TWO_PI;
                else v = (exp(-lo * t) - exp(-hi * t)) / (OR_TWO_PI * t);
            }
            K[(size_t)j * n_tau + i] = v;
        }
    }
    return 0;
}

/* F_i = sum_j K_ji a_j, j ascending (Eq. correlation-model). */
void or_forward(const double *K, int n_omega, int n_tau, const double *a, double *F)
{
    for (int i = 0; i < n_tau; ++i) {
        double s = 0.0;
        for (int j = 0; j < n_omega; ++j) s += K[(size_t)j * n_tau + i] * a[j];
        F[i] = s;
    }
}

/* chi^2 = sum_i w_i (F_i - Ft_i)^2 (Eq. residue; w_i = 1 is the paper's form). */
double or_chi2(const double *F, const double *Ft, const double *w, int n_tau)
{
    double s = 0.0;
    for (int i = 0; i < n_tau; ++i) {
        double r = F[i] - Ft[i];
        s += w[i] * r * r;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Two-parameter renormalisation restoring sum_j a_j = A and                */
/* sum_j a_j omega_j = B (Sec. 2.6 asks for a renormalisation of the second */
/* sum rule after smoothing).  Reading: a_j <- a_j (1 + d0 + d1 omega_j),   */
/* the smallest multiplicative correction linear in omega that fixes both.  */
/* ------------------------------------------------------------------------ */
void or_renormalize(double *a, const double *omega, int n, double A, double B)
{
    double S0 = 0.0, S1 = 0.0, S2 = 0.0;
    for (int j = 0; j < n; ++j) {
        S0 += a[j];
        S1 += a[j] * omega[j];
        S2 += a[j] * omega[j] * omega[j];
    }
    double e0 = A - S0, e1 = B - S1;
    double det = S0 * S2 - S1 * S1;
    if (!(det > 0.0) || !isfinite(det)) return;
    double d0 = (e0 * S2 - e1 * S1) / det;
    double d1 = (e1 * S0 - e0 * S1) / det;
    for (int j = 0; j < n; ++j) a[j] = a[j] + a[j] * (d0 + d1 * omega[j]);
}

/* ------------------------------------------------------------------------ */
/* Smoothing (Sec. 2.6): the three-point stencil with amplitude s,          */
/*   a_j <- s a_{j-1} + (1 - 2s) a_j + s a_{j+1}   for 0 < j < n - 1,        */
/*   a_0 <- (1 - s) a_0 + s a_1,  a_{n-1} <- (1 - s) a_{n-1} + s a_{n-2},   */
/* all on the values before the update.  It keeps sum_j a_j; the second sum */
/* needs the renormalisation above.                                          */
/* ------------------------------------------------------------------------ */
void or_smooth(double *a, int n, double s)
{
    if (n < 2) return;
    const double c = 1.0 - 2.0 * s, e = 1.0 - s;
    double prev = a[0];
    a[0] = e * a[0] + s * a[1];
    for (int j = 1; j < n - 1; ++j) {
        const double cur = a[j];
        a[j] = s * prev + c * cur + s * a[j + 1];
        prev = cur;
    }
    a[n - 1] = e * a[n - 1] + s * prev;
}

/* ------------------------------------------------------------------------ */
/* Initial spectrum.  The paper does not say how walkers start.  Reading:   */
/* the maximum-entropy spectrum that meets both sum rules, a_j ~ e^{-lambda */
/* omega_j}, with lambda found by bisection on the mean frequency B/A, then */
/* scaled to sum A and renormalised.  Returns 1 if B/A lies outside the     */
/* open window (omega_0, omega_{n-1}).                                      */
/* ------------------------------------------------------------------------ */
static double tilt_mean(const double *omega, int n, double lam)
{
    /* shift the exponent so its largest term is exp(0) */
    double ref = lam > 0.0 ? omega[0] : omega[n - 1];
    double s0 = 0.0, s1 = 0.0;
    for (int j = 0; j < n; ++j) {
        double e = exp(-lam * (omega[j] - ref));
        s0 += e;
        s1 += e * omega[j];
    }
    return s1 / s0;
}

int or_init_spectrum(const double *omega, int n, double A, double B, double *a, double *lambda_out)
{
    double mu = B / A;
    if (!(A > 0.0) || !(mu > omega[0]) || !(mu < omega[n - 1])) return 1;
    double lo = -1.0, hi = 1.0; /* tilt_mean is decreasing in lambda */
    for (int it = 0; it < 4000 && tilt_mean(omega, n, lo) <= mu; ++it) lo *= 2.0;
    for (int it = 0; it < 4000 && tilt_mean(omega, n, hi) >= mu; ++it) hi *= 2.0;
    for (int it = 0; it < 300; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (tilt_mean(omega, n, mid) > mu) lo = mid; else hi = mid;
    }
    double lam = 0.5 * (lo + hi);
    if (fabs(tilt_mean(omega, n, 0.0) - mu) <= 0.0) lam = 0.0;
    double ref = lam > 0.0 ? omega[0] : omega[n - 1];
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
        a[j] = exp(-lam * (omega[j] - ref));
        s += a[j];
    }
    for (int j = 0; j < n; ++j) a[j] = a[j] * (A / s);
    or_renormalize(a, omega, n, A, B);
    if (lambda_out) *lambda_out = lam;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Imprinted branching, Sec. 2.5.                                           */
/* Weight w = exp[-(chi^2 - P_r) Delta] (the printed "P(chi^2)" is read as  */
/* chi^2; dividing by T is absorbed into Delta), multiplier                 */
/* m = floor(w + xi).  m_l reaches k once P_r >= theta_{l,k} with           */
/*   theta_{l,k} = chi^2_l + ln(k - xi_l)/Delta,   k = 1, 2, ...            */
/* so sum_l m_l = n exactly when P_r sits between the n-th and (n+1)-th     */
/* smallest threshold (Reading: the midpoint).  Delta is the smallest value */
/* (from a fixed doubling + bisection search) whose zero count reaches      */
/* round(fraction * n).                                                      */
/* ------------------------------------------------------------------------ */
typedef struct { double th; int l; int k; } or_heap_item;

static void heap_push(or_heap_item *h, int *sz, or_heap_item it)
{
    int i = (*sz)++;
    h[i] = it;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (h[p].th <= h[i].th) break;
        or_heap_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static or_heap_item heap_pop(or_heap_item *h, int *sz)
{
    or_heap_item top = h[0];
    h[0] = h[--(*sz)];
    int i = 0;
    for (;;) {
        int c = 2 * i + 1;
        if (c >= *sz) break;
        if (c + 1 < *sz && h[c + 1].th < h[c].th) c = c + 1;
        if (h[i].th <= h[c].th) break;
        or_heap_item t = h[c]; h[c] = h[i]; h[i] = t;
        i = c;
    }
    return top;
}

static double threshold(const double *chi2, const double *xi, int l, int k, double delta)
{
    return chi2[l] + log((double)k - xi[l]) / delta;
}

/* Evaluate the multipliers for a given Delta.  Returns the zero count and sets
 * *pr, m[], *tie (1 when the n-th and (n+1)-th thresholds coincide) and
 * *gap, the distance between those two thresholds relative to the larger of
 * their magnitudes and 1/Delta (the scale of their rounding): how far the
 * multipliers are from changing under a perturbation of the residues. */
static int branch_eval(int n, const double *chi2, const double *xi, double delta,
                       or_heap_item *heap, int32_t *m, double *pr, int *tie, double *gap)
{
    int sz = 0;
    for (int l = 0; l < n; ++l) {
        or_heap_item it = {threshold(chi2, xi, l, 1, delta), l, 1};
        heap_push(heap, &sz, it);
        m[l] = 0;
    }
    double last = 0.0;
    for (int c = 0; c < n; ++c) {
        or_heap_item it = heap_pop(heap, &sz);
        m[it.l] += 1;
        last = it.th;
        or_heap_item nx = {threshold(chi2, xi, it.l, it.k + 1, delta), it.l, it.k + 1};
        heap_push(heap, &sz, nx);
    }
    double next = heap[0].th;
    *tie = (next == last);
    *pr = 0.5 * (last + next);
    double scale = fmax(fmax(fabs(last), fabs(next)), 1.0 / delta);
    *gap = (next - last) / scale;
    int z = 0;
    for (int l = 0; l < n; ++l) z += (m[l] == 0);
    return z;
}

/* Returns 0 on success (m[] set, sum m = n), 1 when the event is skipped
 * (target zero count unreachable or degenerate ensemble); then m[] = 1.
 * Optional margins (NULL skips): *gap_out the threshold gap (branch_eval) at
 * the final Delta (small by construction: the search ends just above the
 * crossing of two thresholds that moves the zero count), *bracket_out the
 * final bracket's relative width (hi - lo) / hi: that crossing lies within
 * it below Delta. */
int or_branch_solve(int n, const double *chi2, const double *xi, double fraction,
                    double *delta_out, double *pr_out, int32_t *m, int *z_out, int *tie_out,
                    double *gap_out, double *bracket_out)
{
    int zt = (int)floor(fraction * (double)n + 0.5);
    double cmin = chi2[0], cmax = chi2[0];
    for (int l = 1; l < n; ++l) {
        if (chi2[l] < cmin) cmin = chi2[l];
        if (chi2[l] > cmax) cmax = chi2[l];
    }
    for (int l = 0; l < n; ++l) m[l] = 1;
    *delta_out = 0.0; *pr_out = 0.0; *z_out = 0; *tie_out = 0;
    if (gap_out) *gap_out = INFINITY;
    if (bracket_out) *bracket_out = INFINITY;
    if (zt <= 0 || zt >= n || !(cmax > cmin) || !isfinite(cmax - cmin)) return 1;
    or_heap_item *heap = (or_heap_item *)malloc(sizeof(or_heap_item) * (size_t)(n + 1));
    int32_t *mt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double pr, gap; int tie;
    double d0 = 1.0 / (cmax - cmin), lo, hi;
    int ok = 1;
#define EVAL(d) branch_eval(n, chi2, xi, (d), heap, mt, &pr, &tie, &gap)
    if (EVAL(d0) >= zt) {
        hi = d0; lo = 0.5 * d0;
        int it = 0;
        while (EVAL(lo) >= zt) {
            hi = lo; lo = 0.5 * lo;
            if (++it >= 200) { ok = 0; break; }
        }
    } else {
        lo = d0; hi = 2.0 * d0;
        int it = 0;
        while (EVAL(hi) < zt) {
            lo = hi; hi = 2.0 * hi;
            if (++it >= 200) { ok = 0; break; }
        }
    }
    if (ok) {
        for (int it = 0; it < 30; ++it) {
            double mid = sqrt(lo * hi);
            if (EVAL(mid) >= zt) hi = mid; else lo = mid;
        }
        int z = EVAL(hi);
        for (int l = 0; l < n; ++l) m[l] = mt[l];
        *delta_out = hi; *pr_out = pr; *z_out = z; *tie_out = tie;
        if (gap_out) *gap_out = gap;
        if (bracket_out) *bracket_out = (hi - lo) / hi;
    }
#undef EVAL
    free(heap);
    free(mt);
    return ok ? 0 : 1;
}

/* Whether the solve's outcome (status and multipliers m_ref) survives a
 * relative perturbation eps of the residues in four sign patterns (all up,
 * all down, alternating, alternating reversed): 1 if every perturbed solve
 * gives the same result.  Residues computed in another arithmetic agree with
 * these only to some relative eps, so a solve that is not robust at that
 * eps may legitimately end with other multipliers there (a near-tie). */
int or_branch_robust(int n, const double *chi2, const double *xi, double fraction, int status_ref,
                     const int32_t *m_ref, double eps)
{
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *m = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int same = 1;
    for (int pat = 0; pat < 4 && same; ++pat) {
        for (int l = 0; l < n; ++l) {
            double sg = (pat == 0) ? 1.0 : (pat == 1) ? -1.0 : ((l & 1) ? -1.0 : 1.0) * (pat == 2 ? 1.0 : -1.0);
            c[l] = chi2[l] * (1.0 + sg * eps);
        }
        double d, pr; int z, tie;
        int st = or_branch_solve(n, c, xi, fraction, &d, &pr, m, &z, &tie, NULL, NULL);
        if (st == 0 && tie) st = 2;
        if (st != 0) for (int l = 0; l < n; ++l) m[l] = 1;
        if (st != status_ref) same = 0;
        for (int l = 0; l < n && same; ++l) same = (m[l] == m_ref[l]);
    }
    free(c);
    free(m);
    return same;
}

/* Pairing (Reading: the paper does not fix it): zero-multiplier walkers in
 * ascending index order meet the donors in ascending index order, donor l
 * repeated m_l - 1 times.  Returns the number of pairs. */
int or_branch_pairs(int n, const int32_t *m, int32_t *targets, int32_t *donors)
{
    int nt = 0, nd = 0;
    for (int l = 0; l < n; ++l) if (m[l] == 0) targets[nt++] = l;
    for (int l = 0; l < n; ++l) for (int c = 1; c < m[l]; ++c) donors[nd++] = l;
    return nt == nd ? nt : -1;
}

/* ------------------------------------------------------------------------ */
/* Eqs. (update-delta-p/s), Sec. 2.2: with a_j' = r a_j for j != p, s and   */
/* a_p' = r a_p + dp, a_s' = r a_s + ds, both sums stay fixed when          */
/*   dp (omega_p - omega_s) = [B - A omega_s] (1 - r),                      */
/*   ds (omega_s - omega_p) = [B - A omega_p] (1 - r)                       */
/* (omega are bin centres, i.e. the paper's omega + d_omega/2).  p == s has */
/* no solution; the deltas are then zero and the proposal is rejected.     */
/* ------------------------------------------------------------------------ */
void or_move_deltas(const double *omega, double A, double B, int p, int s, double r, double *dp, double *ds)
{
    double omr = 1.0 - r;
    if (p == s) { *dp = 0.0; *ds = 0.0; return; }
    *dp = omr * (B - A * omega[s]) / (omega[p] - omega[s]);
    *ds = omr * (B - A * omega[p]) / (omega[s] - omega[p]);
}

/* ------------------------------------------------------------------------ */
/* The anneal.                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    /* problem */
    int n_omega, n_tau, n_walkers;
    const double *omega, *Ft, *w, *K; /* K is [n_omega][n_tau] */
    double A, B;
    /* schedule: temperature of global sweep k is T[k] * chi2_unit */
    const double *T;
    int n_T;
    double chi2_unit;
    int branch_every, resync_every;
    double branch_fraction, imprint_t, eps0, amp_p, amp_avg;
    int amp_m, walk_len;
    uint64_t seed;
    /* optional per-proposal trace over sweeps [trace_k0, trace_k1), layout
     * [walker][sweep - trace_k0][proposal]; any pointer may be NULL */
    int trace_k0, trace_k1;
    double *trace_dchi2, *trace_cond;
    uint8_t *trace_accept;
    /* optional decisions taken elsewhere (same layout).  Where a decision
     * differs from the oracle's own and the oracle's margin lies inside the
     * near-tie band, the other decision is adopted; outside the band the
     * oracle keeps its own and counts a hard mismatch. */
    const uint8_t *replay_accept;
    double band;
    /* optional branching log, indexed by absolute event number */
    int max_events;
    double *ev_delta, *ev_pr;
    int32_t *ev_z, *ev_status, *ev_m; /* ev_m is [event][walker] */
    /* optional global walker numbers of the rows held here (NULL: row l is
     * walker l); lets a test replay a sample of a large population.  Only
     * valid for stretches without a branching event. */
    const int32_t *walker_ids;
    /* results */
    int64_t n_near_ties, n_hard_mismatch, n_proposals, n_accepted;
    int32_t first_mismatch[3]; /* walker, sweep, proposal of the earliest hard mismatch, or -1 */
    /* optional: the two bins each traced proposal chose (after the
     * selection walk), same layout as the other traces */
    int32_t *trace_p, *trace_s;
    /* smoothing amplitude s of Sec. 2.6 (0: none).  Reading: after every
     * branching event each walker is smoothed, renormalised, and its F and
     * chi^2 recomputed, so the next block's sweeps start from smoothed
     * spectra */
    double smooth;
    /* adaptive branching (Sec. 2.5, last paragraph).  Reading: at each event
     * the branching fraction and the imprint strength are scaled by the
     * population mean of the running acceptance rate (which starts at 1) */
    int adaptive;
    /* self-cooling (Sec. 2.4).  Reading: the temperature of block b (all its
     * sweeps) follows from the population's residues at the block's start:
     * boil (b < boil_blocks) T = mean chi^2; cool (the next cool_blocks
     * blocks) T = (1 - x) mean + x min with x = (b - boil_blocks + 1) /
     * cool_blocks; freeze (after) T = min / (1 + j), j the freeze block
     * count from 1.  The mean sums the walkers in order.  The temperatures
     * used are written to T_self[k] (absolute units; n_T entries). */
    int self_cool, boil_blocks, cool_blocks;
    double *T_self;
    /* optional branching margins per event (or_branch_solve): the threshold
     * gap at the final Delta and the final bracket width; and whether the
     * event is robust (or_branch_robust at branch_band) */
    double *ev_gap, *ev_bracket;
    int32_t *ev_robust;
    /* optional multipliers taken elsewhere, [event][walker] for events
     * [0, replay_m_events).  Where they differ from the oracle's own and the
     * event is not robust to a relative perturbation branch_band of the
     * residues (a branching near-tie), they are adopted; otherwise the oracle
     * keeps its own and counts a hard branching mismatch. */
    const int32_t *replay_m;
    int replay_m_events;
    double branch_band;
    int64_t n_branch_near_ties, n_branch_hard;
    int32_t first_branch_mismatch; /* event of the earliest hard branching mismatch, or -1 */
} or_anneal_args;

typedef struct { int64_t near, hard, props, acc; int32_t fk, fq; } walker_log;

/* Sweeps [k0, k1) of one walker.  Sec. 2.2 (moves, Eqs. update-scheme and
 * update-delta, incremental F'), Sec. 2.3 (uniform selection for zero walk
 * length, Markov walk on a_j / A otherwise), Sec. 2.7 (amplitude factor y),
 * Eq. (probability-density) for the Metropolis test. */
static void walker_sweeps(const or_anneal_args *g, int l, int k0, int k1,
                          double *a, double *F, double *chi2, double *rate,
                          double *dF, walker_log *lg)
{
    const int No = g->n_omega, Nt = g->n_tau;
    const double *omega = g->omega, *K = g->K, *w = g->w, *Ft = g->Ft;
    const uint32_t gl = g->walker_ids ? (uint32_t)g->walker_ids[l] : (uint32_t)l;
    for (int k = k0; k < k1; ++k) {
        double Tabs = g->self_cool ? g->T_self[k] : g->T[k] * g->chi2_unit;
        /* Eq. (amplitude-acceptance-adjustment).  Reading: the "ongoing"
         * acceptance rate is a running average over sweeps,
         *   rate <- (1 - amp_avg) rate + amp_avg (accepted / n_omega),
         * starting from 1 (amp_avg = 1 is the previous sweep alone). */
        double y = 1.0;
        if (*rate < g->amp_p) {
            double q = *rate / g->amp_p;
            for (int c = 0; c < g->amp_m; ++c) y = y * q;
        }
        int32_t acc = 0;
        int traced = (k >= g->trace_k0 && k < g->trace_k1);
        size_t toff = traced ? ((size_t)l * (size_t)(g->trace_k1 - g->trace_k0) + (size_t)(k - g->trace_k0)) * (size_t)No : 0;
        for (int q = 0; q < No; ++q) {
            uint32_t x[4];
            draw(g->seed, (uint32_t)q, (uint32_t)k, gl, OR_STREAM_PROPOSAL, x);
            int p = index_of(x[0], No), s = index_of(x[1], No);
            /* Sec. 2.3: truncated independence walk on P(j) = a_j / A */
            for (int st = 1; st <= g->walk_len; ++st) {
                uint32_t y4[4];
                draw(g->seed, (uint32_t)q, (uint32_t)k, gl, (uint32_t)st, y4);
                int pc = index_of(y4[0], No), sc = index_of(y4[2], No);
                if (u01(y4[1]) * a[p] < a[pc]) p = pc;
                if (u01(y4[3]) * a[s] < a[sc]) s = sc;
            }
            double ur = u01(x[2]), ua = u01(x[3]);
            double r = 1.0 - y * g->eps0 * (2.0 * ur - 1.0);
            double rm1 = r - 1.0;
            double dp, ds;
            or_move_deltas(omega, g->A, g->B, p, s, r, &dp, &ds);
            double ap = r * a[p] + dp, as = r * a[s] + ds;
            int ok = (p != s) && ap >= 0.0 && as >= 0.0;
            /* Sec. 2.2: F' = r F + dp K_p + ds K_s, so dF costs O(N_tau). */
            double d = 0.0;
            for (int i = 0; i < Nt; ++i) {
                double f = rm1 * F[i] + dp * K[(size_t)p * Nt + i] + ds * K[(size_t)s * Nt + i];
                dF[i] = f;
                d += w[i] * f * (2.0 * (F[i] - Ft[i]) + f);
            }
            int accept = ok && (d <= 0.0 || ua < exp(-d / Tabs));
            if (traced && (g->trace_dchi2 || g->trace_cond || g->replay_accept)) {
                /* condition scale of the d computation: every term taken in
                 * absolute value, the residual bounded through |F| + |Ft| */
                double M = 0.0;
                for (int i = 0; i < Nt; ++i) {
                    double mag = fabs(rm1) * fabs(F[i]) + fabs(dp) * K[(size_t)p * Nt + i] + fabs(ds) * K[(size_t)s * Nt + i];
                    M += w[i] * mag * (2.0 * fabs(F[i]) + 2.0 * fabs(Ft[i]) + fabs(dF[i]));
                }
                if (g->trace_dchi2) g->trace_dchi2[toff + q] = d;
                if (g->trace_cond) g->trace_cond[toff + q] = M;
                if (g->replay_accept) {
                    int other = (g->replay_accept[toff + q] & 1) != 0;
                    if (other != accept) {
                        int near = 0;
                        double b = g->band;
                        if (p != s) {
                            if (fabs(ap) <= b * (fabs(r * a[p]) + fabs(dp))) near = 1;
                            if (fabs(as) <= b * (fabs(r * a[s]) + fabs(ds))) near = 1;
                        }
                        if (ok) {
                            if (fabs(d) <= b * M) near = 1;
                            if (d > 0.0) {
                                double e = exp(-d / Tabs);
                                if (fabs(ua - e) <= e * (b * M / Tabs + 1e-13)) near = 1;
                            }
                        }
                        if (near) {
                            lg->near++;
                            accept = other;
                        } else {
                            if (lg->hard == 0) { lg->fk = k; lg->fq = q; }
                            lg->hard++;
                        }
                    }
                }
            }
            if (traced && g->trace_p) g->trace_p[toff + q] = p;
            if (traced && g->trace_s) g->trace_s[toff + q] = s;
            /* bit 0: accepted, bit 1: move admissible (p != s and a' >= 0) */
            if (traced && g->trace_accept) g->trace_accept[toff + q] = (uint8_t)(accept | (ok << 1));
            lg->props++;
            if (accept) {
                /* Eqs. (update-scheme-p/s/j): every coefficient scales by r,
                 * the two chosen ones also receive their delta. */
                for (int j = 0; j < No; ++j) a[j] = r * a[j];
                a[p] = ap;
                a[s] = as;
                for (int i = 0; i < Nt; ++i) F[i] = F[i] + dF[i];
                *chi2 = *chi2 + d;
                acc++;
                lg->acc++;
            }
        }
        *rate = (1.0 - g->amp_avg) * (*rate) + g->amp_avg * ((double)acc / (double)No);
    }
}

/* Exact recomputation after sweeps whose count is a multiple of
 * resync_every: renormalise the two sums, then F = K a and chi^2 afresh. */
static void resync_walker(const or_anneal_args *g, double *a, double *F, double *chi2)
{
    or_renormalize(a, g->omega, g->n_omega, g->A, g->B);
    or_forward(g->K, g->n_omega, g->n_tau, a, F);
    *chi2 = or_chi2(F, g->Ft, g->w, g->n_tau);
}

/* One branching event (Sec. 2.5): xi_l from the branching stream, solve,
 * pair, imprint a^(l1) <- t a^(l2) + (1 - t) a^(l1), recompute F, chi^2.
 * With adaptive branching the fraction and t are scaled by the mean rate. */
static int branch_event(or_anneal_args *g, int e, double *a, double *F, double *chi2, const double *rate)
{
    const int n = g->n_walkers, No = g->n_omega, Nt = g->n_tau;
    double *xi = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *m = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *tg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dn = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int l = 0; l < n; ++l) {
        uint32_t x[4];
        draw(g->seed, (uint32_t)l, (uint32_t)e, 0u, OR_STREAM_BRANCH, x);
        xi[l] = u01(x[0]);
    }
    double fraction = g->branch_fraction, t = g->imprint_t;
    if (g->adaptive) {
        double mean = 0.0;
        for (int l = 0; l < n; ++l) mean += rate[l];
        mean /= (double)n;
        fraction *= mean;
        t *= mean;
    }
    double delta, pr, gap, bracket; int z, tie;
    int st = or_branch_solve(n, chi2, xi, fraction, &delta, &pr, m, &z, &tie, &gap, &bracket);
    if (st == 0 && tie) st = 2; /* A tie leaves sum m = n ambiguous: skip. */
    if (st != 0) for (int l = 0; l < n; ++l) m[l] = 1;
    int robust = -1; /* not evaluated */
    if (g->ev_robust || g->replay_m) robust = or_branch_robust(n, chi2, xi, fraction, st, m, g->branch_band);
    int adopted = 0;
    if (g->replay_m && e < g->replay_m_events) {
        const int32_t *mr = g->replay_m + (size_t)e * n;
        int differ = 0;
        int64_t sum = 0;
        for (int l = 0; l < n; ++l) { differ |= (mr[l] != m[l]); sum += mr[l]; }
        if (differ) {
            if (!robust && sum == n) {
                memcpy(m, mr, sizeof(int32_t) * (size_t)n);
                adopted = 1;
                g->n_branch_near_ties++;
            } else {
                g->n_branch_hard++;
                if (g->first_branch_mismatch < 0) g->first_branch_mismatch = e;
            }
        }
    }
    if (g->ev_status && e < g->max_events) {
        g->ev_status[e] = st;
        if (g->ev_delta) g->ev_delta[e] = delta;
        if (g->ev_pr) g->ev_pr[e] = pr;
        if (g->ev_z) g->ev_z[e] = z;
        if (g->ev_m) memcpy(g->ev_m + (size_t)e * n, m, sizeof(int32_t) * (size_t)n);
        if (g->ev_gap) g->ev_gap[e] = gap;
        if (g->ev_bracket) g->ev_bracket[e] = bracket;
        if (g->ev_robust) g->ev_robust[e] = robust;
    }
    if (st == 0 || adopted) {
        int np = or_branch_pairs(n, m, tg, dn);
        for (int c = 0; c < np; ++c) {
            double *a1 = a + (size_t)tg[c] * No;
            const double *a2 = a + (size_t)dn[c] * No;
            for (int j = 0; j < No; ++j) a1[j] = t * a2[j] + (1.0 - t) * a1[j];
            or_forward(g->K, No, Nt, a1, F + (size_t)tg[c] * Nt);
            chi2[tg[c]] = or_chi2(F + (size_t)tg[c] * Nt, g->Ft, g->w, Nt);
        }
    }
    free(xi); free(m); free(tg); free(dn);
    return st;
}

/* Self-cooling temperature of block b from the current residues. */
static double self_cool_T(const or_anneal_args *g, int b, const double *chi2)
{
    double sum = 0.0, mn = chi2[0];
    for (int l = 0; l < g->n_walkers; ++l) {
        sum += chi2[l];
        if (chi2[l] < mn) mn = chi2[l];
    }
    const double mean = sum / (double)g->n_walkers;
    if (b < g->boil_blocks) return mean;
    if (b < g->boil_blocks + g->cool_blocks) {
        const double x = (double)(b - g->boil_blocks + 1) / (double)g->cool_blocks;
        return (1.0 - x) * mean + x * mn;
    }
    return mn / (double)(1 + (b - g->boil_blocks - g->cool_blocks + 1));
}

/* Runs global sweeps [k0, k1).  State arrays are [walker][...] and are
 * updated in place.  After sweep k, if (k+1) % resync_every == 0 every walker
 * is resynced, and if (k+1) % branch_every == 0 branching event
 * (k+1)/branch_every - 1 follows.  Walkers are independent between those
 * points, so the loop over walkers may run on several threads. */
int or_anneal(or_anneal_args *g, int k0, int k1, double *a, double *F, double *chi2, double *rate)
{
    const int n = g->n_walkers, No = g->n_omega, Nt = g->n_tau;
    if (k0 < 0 || k1 > g->n_T || k0 > k1) return 1;
    if (g->resync_every <= 0 || g->branch_every <= 0 || g->branch_every % g->resync_every != 0) return 1;
    if (g->walker_ids && k1 / g->branch_every > k0 / g->branch_every) return 2;
    if (g->walker_ids && g->self_cool) return 2; /* needs the whole population */
    walker_log *lg = (walker_log *)calloc((size_t)n, sizeof(walker_log));
    for (int l = 0; l < n; ++l) { lg[l].fk = -1; lg[l].fq = -1; }
    int k = k0;
    while (k < k1) {
        if (g->self_cool && k % g->branch_every == 0) {
            const double Tb = self_cool_T(g, k / g->branch_every, chi2);
            for (int q = k; q < k + g->branch_every && q < g->n_T; ++q) g->T_self[q] = Tb;
        }
        int kend = ((k / g->resync_every) + 1) * g->resync_every;
        if (kend > k1) kend = k1;
#pragma omp parallel
        {
            double *dF = (double *)malloc(sizeof(double) * (size_t)Nt);
#pragma omp for schedule(dynamic, 1)
            for (int l = 0; l < n; ++l)
                walker_sweeps(g, l, k, kend, a + (size_t)l * No, F + (size_t)l * Nt, chi2 + l, rate + l, dF, lg + l);
            free(dF);
        }
        if (kend % g->resync_every == 0) {
#pragma omp parallel for schedule(static)
            for (int l = 0; l < n; ++l) resync_walker(g, a + (size_t)l * No, F + (size_t)l * Nt, chi2 + l);
        }
        if (kend % g->branch_every == 0) {
            branch_event(g, kend / g->branch_every - 1, a, F, chi2, rate);
            if (g->smooth > 0.0) {
#pragma omp parallel for schedule(static)
                for (int l = 0; l < n; ++l) {
                    or_smooth(a + (size_t)l * No, No, g->smooth);
                    resync_walker(g, a + (size_t)l * No, F + (size_t)l * Nt, chi2 + l);
                }
            }
        }
        k = kend;
    }
    int64_t near = 0, hard = 0, props = 0, acc = 0;
    g->first_mismatch[0] = g->first_mismatch[1] = g->first_mismatch[2] = -1;
    for (int l = 0; l < n; ++l) {
        near += lg[l].near; hard += lg[l].hard; props += lg[l].props; acc += lg[l].acc;
        if (lg[l].hard > 0) {
            int better = g->first_mismatch[0] < 0 || lg[l].fk < g->first_mismatch[1] ||
                         (lg[l].fk == g->first_mismatch[1] && lg[l].fq < g->first_mismatch[2]);
            if (better) { g->first_mismatch[0] = l; g->first_mismatch[1] = lg[l].fk; g->first_mismatch[2] = lg[l].fq; }
        }
    }
    g->n_near_ties += near; g->n_hard_mismatch += hard; g->n_proposals += props; g->n_accepted += acc;
    free(lg);
    return 0;
}

/* Walker set-up: every walker starts from the same spectrum a0 (Reading: the
 * paper does not say), with F = K a0, its chi^2, and an acceptance rate of 1
 * so the first sweep uses y = 1. */
void or_walkers_init(const or_anneal_args *g, const double *a0, double *a, double *F, double *chi2, double *rate)
{
    const int n = g->n_walkers, No = g->n_omega, Nt = g->n_tau;
    double *F0 = (double *)malloc(sizeof(double) * (size_t)Nt);
    or_forward(g->K, No, Nt, a0, F0);
    double c0 = or_chi2(F0, g->Ft, g->w, Nt);
    for (int l = 0; l < n; ++l) {
        memcpy(a + (size_t)l * No, a0, sizeof(double) * (size_t)No);
        memcpy(F + (size_t)l * Nt, F0, sizeof(double) * (size_t)Nt);
        chi2[l] = c0;
        rate[l] = 1.0;
    }
    free(F0);
}

/* Ensemble-averaged spectrum, Eq. (residue-average) estimated over walkers. */
void or_mean_spectrum(int n_walkers, int n_omega, const double *a, double *out)
{
    for (int j = 0; j < n_omega; ++j) {
        double s = 0.0;
        for (int l = 0; l < n_walkers; ++l) s += a[(size_t)l * n_omega + j];
        out[j] = s / (double)n_walkers;
    }
}

/* Histogram of log10 chi^2 over [lo, hi) in n_bins equal bins; values
 * outside are clamped into the end bins. */
void or_chi2_hist(int n, const double *chi2, int n_bins, double lo, double hi, uint64_t *counts)
{
    for (int b = 0; b < n_bins; ++b) counts[b] = 0;
    double width = hi - lo;
    for (int l = 0; l < n; ++l) {
        double v = log10(chi2[l]);
        int b = (width > 0.0) ? (int)floor((v - lo) / width * (double)n_bins) : 0;
        if (!(v == v)) b = 0;
        if (b < 0) b = 0;
        if (b >= n_bins) b = n_bins - 1;
        counts[b]++;
    }
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads later calls use (n >= 1). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
