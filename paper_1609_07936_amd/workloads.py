"""Seeded synthetic inputs for the annealing inverse Laplace transform.

This module only builds inputs: frequency and time grids, a target spectrum
made of truncated Lorentzians, its transform F(tau) by quadrature, its first
two moments, and Gaussian noise.  It holds none of the method's arithmetic
(no model kernel table, no residue, no moves), so the GPU library and the
CPU oracle can both take their inputs from here.

Target family (Sec. 5.2 of the paper uses a two-peak Lorentzian band):
    S(omega) = sum_k c_k L(omega; omega_k, Gamma_k)  on  [0, omega_max],
    L(omega; omega_0, Gamma) = (Gamma/pi) / ((omega - omega_0)^2 + Gamma^2),
truncated to the model window and renormalised to unit zeroth moment.
The transform is F(tau) = (1/2pi) int_0^omega_max S(omega) e^{-omega tau} d omega
(Eq. transform), evaluated by composite Simpson on 1e5 intervals.
Noise is iid Gaussian with sigma_i = level * F_i, or, for the paper's band
workload, the correlated undersampling noise of Sec. 5.1 (resampled_data).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TWO_PI = 2.0 * np.pi


def lorentzian(w, w0: float, gamma: float):
    return (gamma / np.pi) / ((w - w0) ** 2 + gamma ** 2)


def lorentzian_mass(w0: float, gamma: float, lo: float, hi: float) -> float:
    """int_lo^hi L(omega; w0, gamma) d omega in closed form."""
    return float((np.arctan((hi - w0) / gamma) - np.arctan((lo - w0) / gamma)) / np.pi)


@dataclass
class Target:
    """Sum of Lorentzians on the support [lo, hi] (default the whole window
    [0, omega_max]; Eq. lorentzian-band clips to a band), unit zeroth moment."""
    centres: np.ndarray
    widths: np.ndarray
    weights: np.ndarray
    omega_max: float
    lo: float = 0.0
    hi: float | None = None

    def __post_init__(self):
        self.centres = np.asarray(self.centres, dtype=np.float64)
        self.widths = np.asarray(self.widths, dtype=np.float64)
        self.weights = np.asarray(self.weights, dtype=np.float64)
        if self.hi is None:
            self.hi = self.omega_max
        mass = sum(c * lorentzian_mass(w0, g, self.lo, self.hi)
                   for c, w0, g in zip(self.weights, self.centres, self.widths))
        self.norm = 1.0 / mass  # unit zeroth moment on the support

    def density(self, w):
        w = np.asarray(w, dtype=np.float64)
        s = np.zeros_like(w)
        for c, w0, g in zip(self.weights, self.centres, self.widths):
            s = s + c * lorentzian(w, w0, g)
        return self.norm * s * ((w >= self.lo) & (w <= self.hi))


def simpson_weights(n_intervals: int, h: float) -> np.ndarray:
    if n_intervals % 2:
        raise ValueError("Simpson needs an even number of intervals")
    wts = np.ones(n_intervals + 1)
    wts[1:-1:2] = 4.0
    wts[2:-1:2] = 2.0
    return wts * (h / 3.0)


def transform_quadrature(target: Target, tau, n_intervals: int = 100_000):
    """F(tau_i), m0 = int S, m1 = int omega S by composite Simpson on the support [lo, hi]."""
    tau = np.asarray(tau, dtype=np.float64)
    h = (target.hi - target.lo) / n_intervals
    x = np.linspace(target.lo, target.hi, n_intervals + 1)
    wq = simpson_weights(n_intervals, h) * target.density(x)
    F = np.array([np.dot(wq, np.exp(-x * t)) for t in tau]) / TWO_PI
    m0 = float(np.sum(wq))
    m1 = float(np.dot(wq, x))
    return F, m0, m1


@dataclass
class Workload:
    name: str
    omega: np.ndarray       # bin centres, uniform
    tau: np.ndarray         # uniform time grid
    F_true: np.ndarray      # noise-free transform
    Ft: np.ndarray          # noisy data
    sigma: np.ndarray       # per-point error
    m0: float
    m1: float
    target: Target
    n_walkers: int
    n_sweeps: int
    t_hi: float
    t_lo: float
    branch_every: int
    resync_every: int
    seed: int               # run seed (Philox key)


def bin_centres(omega_max: float, n_omega: int) -> np.ndarray:
    dw = omega_max / n_omega
    return (np.arange(n_omega, dtype=np.float64) + 0.5) * dw


def uniform_tau(t0: float, t1: float, n_tau: int) -> np.ndarray:
    dt = (t1 - t0) / (n_tau - 1)
    return t0 + dt * np.arange(n_tau, dtype=np.float64)


def make(name: str, omega_max: float, n_omega: int, tau, target: Target, noise: float, data_seed: int,
         n_walkers: int, n_sweeps: int, t_hi: float, t_lo: float, branch_every: int, resync_every: int,
         run_seed: int, n_quad: int = 100_000) -> Workload:
    omega = bin_centres(omega_max, n_omega)
    tau = np.asarray(tau, dtype=np.float64)
    F, m0, m1 = transform_quadrature(target, tau, n_quad)
    rng = np.random.default_rng(data_seed)
    sigma = noise * F
    Ft = F + sigma * rng.standard_normal(F.size)
    return Workload(name, omega, tau, F, Ft, sigma, m0, m1, target, n_walkers, n_sweeps, t_hi, t_lo,
                    branch_every, resync_every, run_seed)


def two_peak_random(rng: np.random.Generator, omega_max: float, n_peaks: int = 2) -> Target:
    centres = rng.uniform(0.5, 8.0, n_peaks)
    widths = rng.uniform(0.05, 1.0, n_peaks)
    if n_peaks == 2:
        w = rng.uniform(0.0, 1.0)
        weights = np.array([w, 1.0 - w])
    else:
        weights = rng.dirichlet(np.ones(n_peaks))
    return Target(centres, widths, weights, omega_max)


def small_64x32(n_sweeps: int = 2000, n_walkers: int = 64) -> Workload:
    """64 bins on [0, 10], 32 times on [0.05, 1.6], 0.6 L(1.5, 0.2) + 0.4 L(4, 0.5),
    noise 1e-4 F, 64 walkers, T 1e2 -> 1e-3 over 2000 sweeps, blocks of 100."""
    tgt = Target([1.5, 4.0], [0.2, 0.5], [0.6, 0.4], 10.0)
    return make("small-64x32", 10.0, 64, uniform_tau(0.05, 1.6, 32), tgt, 1e-4, 1, n_walkers, n_sweeps,
                1e2, 1e-3, 100, 100, 1)


def large_512x128(data_seed: int = 2, n_sweeps: int = 20000, n_walkers: int = 16384,
                  resync_every: int = 100) -> Workload:
    """512 bins on [0, 20], 128 times on [0.02, 3], two seeded Lorentzians
    (centres U[0.5, 8], half-widths U[0.05, 1], weights w, 1-w), noise 1e-5 F,
    16384 walkers, T 1e3 -> 1e-2 over 20000 sweeps, blocks of 100."""
    rng = np.random.default_rng(data_seed)
    tgt = two_peak_random(rng, 20.0, 2)
    return make("large-512x128", 20.0, 512, uniform_tau(0.02, 3.0, 128), tgt, 1e-5, data_seed, n_walkers, n_sweeps,
                1e3, 1e-2, 100, resync_every, data_seed)


def large_512x128_fp32(data_seed: int = 2, n_sweeps: int = 20000, n_walkers: int = 16384) -> Workload:
    """large_512x128 for the FP32 residual loop: resync every 50 sweeps."""
    wl = large_512x128(data_seed, n_sweeps, n_walkers, resync_every=50)
    wl.name = "large-512x128-fp32"
    return wl


def batch_jobs(n_jobs: int = 256, base_seed: int = 1000, n_sweeps: int = 1000) -> list[Workload]:
    """Jobs of the mixed-size batch workload: N_omega in {128..1024} on [0, 20], N_tau in
    {32..256} on [0.02, 3], walkers in {256, 1024, 4096}, 2-3 peaks, noise
    log-uniform in [1e-6, 1e-3]."""
    jobs = []
    for idx in range(n_jobs):
        rng = np.random.default_rng(base_seed + idx)
        n_omega = int(rng.choice([128, 256, 512, 1024]))
        n_tau = int(rng.choice([32, 64, 128, 256]))
        n_walkers = int(rng.choice([256, 1024, 4096]))
        n_peaks = int(rng.choice([2, 3]))
        tgt = two_peak_random(rng, 20.0, n_peaks)
        noise = float(10.0 ** rng.uniform(-6.0, -3.0))
        jobs.append(make(f"job{idx}", 20.0, n_omega, uniform_tau(0.02, 3.0, n_tau), tgt, noise,
                         base_seed + idx, n_walkers, n_sweeps, 1e3, 1e-2, 100, 50, base_seed + idx,
                         n_quad=20_000))
    return jobs


def geometric_schedule(t_hi: float, t_lo: float, n_sweeps: int) -> np.ndarray:
    """T_k = t_hi (t_lo / t_hi)^(k / (S - 1)), in units of the starting residue."""
    if n_sweeps == 1:
        return np.array([t_hi])
    k = np.arange(n_sweeps, dtype=np.float64)
    return t_hi * (t_lo / t_hi) ** (k / (n_sweeps - 1))


def resampled_data(target: Target, tau, n_seq: int, seed: int, n_quad: int = 100_000, chunk: int = 4096):
    """Correlation data with undersampling noise (Sec. 5.1): draw n_seq
    stationary Gaussian sequences on the uniform lag grid whose covariance is
    the exact F(|i - j| d_tau), and estimate F at each lag of tau as the
    sample autocorrelation of the set.  Reading: a sequence holds 2 N_tau
    points, each sequence's estimate averages over all origins, and sigma is
    the standard error of the mean over sequences.  tau must start at 0.
    Returns (F_true, F_estimate, sigma, m0, m1)."""
    tau = np.asarray(tau, dtype=np.float64)
    n_tau = tau.size
    dt = tau[1] - tau[0]
    if abs(tau[0]) > 1e-15 or not np.allclose(np.diff(tau), dt, rtol=1e-12, atol=0):
        raise ValueError("resampled data need a uniform tau grid starting at 0")
    L = 2 * n_tau
    lags = dt * np.arange(L)
    Fl, m0, m1 = transform_quadrature(target, lags, n_quad)
    C = Fl[np.abs(np.arange(L)[:, None] - np.arange(L)[None, :])]
    lam, V = np.linalg.eigh(C)
    A = V * np.sqrt(np.clip(lam, 0.0, None))  # C = A A^T (negative rounding eigenvalues clipped)
    rng = np.random.default_rng(seed)
    counts = (L - np.arange(n_tau)).astype(np.float64)
    s1 = np.zeros(n_tau)
    s2 = np.zeros(n_tau)
    done = 0
    while done < n_seq:
        m = min(chunk, n_seq - done)
        X = rng.standard_normal((m, L)) @ A.T
        Xf = np.fft.rfft(X, 2 * L, axis=1)
        r = np.fft.irfft(Xf * np.conj(Xf), 2 * L, axis=1)[:, :n_tau] / counts
        s1 += r.sum(axis=0)
        s2 += (r * r).sum(axis=0)
        done += m
    est = s1 / n_seq
    var = np.maximum(s2 / n_seq - est * est, 0.0)
    sigma = np.sqrt(var / n_seq)
    return Fl[:n_tau], est, sigma, m0, m1


def paper_band(noise: str = "none", n_seq: int = 0, level: float = 0.0, seed: int = 7, n_omega: int = 1000,
               n_tau: int = 64, d_tau: float = 0.1, n_walkers: int = 1500, n_sweeps: int = 20000) -> Workload:
    """The paper's model (Eq. lorentzian-band): L(omega; 1, 1) + L(omega; 2, 1)
    clipped to [0.5, 2.5], n_omega bins on [0, 3.5], 1500 walkers (Sec. 5.3).
    The tau grid is a reading (the paper does not give it): n_tau uniform
    points from 0 in steps of d_tau.  noise: "none" (exact data, unweighted
    residue), "iid" (sigma = level F), or "resampled" (the Sec. 5.1 generator
    with n_seq sequences).  Blocks of 100 sweeps."""
    tgt = Target([1.0, 2.0], [1.0, 1.0], [1.0, 1.0], 3.5, lo=0.5, hi=2.5)
    omega = bin_centres(3.5, n_omega)
    tau = d_tau * np.arange(n_tau, dtype=np.float64)
    if noise == "resampled":
        F, Ft, sigma, m0, m1 = resampled_data(tgt, tau, n_seq, seed)
    else:
        F, m0, m1 = transform_quadrature(tgt, tau)
        if noise == "iid":
            rng = np.random.default_rng(seed)
            sigma = level * F
            Ft = F + sigma * rng.standard_normal(F.size)
        elif noise == "none":
            Ft, sigma = F.copy(), None
        else:
            raise ValueError(f"unknown noise model {noise!r}")
    return Workload(f"band-{noise}", omega, tau, F, Ft, sigma, m0, m1, tgt, n_walkers, n_sweeps, 1.0, 1.0, 100, 100,
                    seed)


def band_skew(spectrum, omega, omega_m: float = 1.5) -> float:
    """The skew of Sec. 5.3: |int_0^omega_m S - int_omega_m^inf S| / int S, the
    bins split by whether their centre lies below omega_m."""
    a = np.asarray(spectrum, dtype=np.float64)
    left = a[np.asarray(omega) < omega_m].sum()
    return float(abs(left - (a.sum() - left)) / a.sum())
