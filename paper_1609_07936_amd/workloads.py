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
Noise is iid Gaussian with sigma_i = level * F_i (the paper draws correlated
noise from resampled sequences; that generator is not reproduced here).
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
    centres: np.ndarray
    widths: np.ndarray
    weights: np.ndarray
    omega_max: float

    def __post_init__(self):
        self.centres = np.asarray(self.centres, dtype=np.float64)
        self.widths = np.asarray(self.widths, dtype=np.float64)
        self.weights = np.asarray(self.weights, dtype=np.float64)
        mass = sum(c * lorentzian_mass(w0, g, 0.0, self.omega_max)
                   for c, w0, g in zip(self.weights, self.centres, self.widths))
        self.norm = 1.0 / mass  # unit zeroth moment on [0, omega_max]

    def density(self, w):
        w = np.asarray(w, dtype=np.float64)
        s = np.zeros_like(w)
        for c, w0, g in zip(self.weights, self.centres, self.widths):
            s = s + c * lorentzian(w, w0, g)
        return self.norm * s * ((w >= 0.0) & (w <= self.omega_max))


def simpson_weights(n_intervals: int, h: float) -> np.ndarray:
    if n_intervals % 2:
        raise ValueError("Simpson needs an even number of intervals")
    wts = np.ones(n_intervals + 1)
    wts[1:-1:2] = 4.0
    wts[2:-1:2] = 2.0
    return wts * (h / 3.0)


def transform_quadrature(target: Target, tau, n_intervals: int = 100_000):
    """F(tau_i), m0 = int S, m1 = int omega S by composite Simpson on [0, omega_max]."""
    tau = np.asarray(tau, dtype=np.float64)
    h = target.omega_max / n_intervals
    x = np.linspace(0.0, target.omega_max, n_intervals + 1)
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
