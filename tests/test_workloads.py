"""Pins of the seeded input generator: quadrature against closed forms."""
import numpy as np
from scipy.special import exp1

from paper_1609_07936_amd import workloads as W


def _closed_F(target, tau):
    """(1/2pi) int_0^Wmax S e^{-omega tau} d omega with each truncated
    Lorentzian done by the complex exponential integral:
    (Gamma/pi)/((omega-c)^2+Gamma^2) = Im[1/(omega - z)]/pi, z = c + i Gamma,
    and int_0^W e^{-omega tau}/(omega - z) = e^{-z tau}[E1(-z tau) - E1((W - z) tau)]."""
    tau = np.asarray(tau, dtype=np.float64)
    tot = np.zeros_like(tau)
    for c, w0, g in zip(target.weights, target.centres, target.widths):
        z = complex(w0, g)
        val = np.exp(-z * tau) * (exp1(-z * tau) - exp1((target.omega_max - z) * tau))
        tot += c * np.imag(val) / np.pi
    return target.norm * tot / (2 * np.pi)


def _closed_m1(target):
    W_ = target.omega_max
    tot = 0.0
    for c, w0, g in zip(target.weights, target.centres, target.widths):
        tot += c * ((g / (2 * np.pi)) * np.log(((W_ - w0) ** 2 + g ** 2) / (w0 ** 2 + g ** 2))
                    + w0 * W.lorentzian_mass(w0, g, 0.0, W_))
    return target.norm * tot


def test_small_quadrature_matches_exponential_integral():
    wl = W.small_64x32()
    ref = _closed_F(wl.target, wl.tau)
    np.testing.assert_allclose(wl.F_true, ref, rtol=1e-12)
    assert abs(wl.m0 - 1.0) < 1e-12
    assert abs(wl.m1 - _closed_m1(wl.target)) < 1e-11


def test_small_grids_and_noise():
    wl = W.small_64x32()
    assert wl.omega.size == 64 and abs(wl.omega[1] - wl.omega[0] - 0.15625) < 1e-15
    assert abs(wl.omega[0] - 0.078125) < 1e-15
    assert wl.tau.size == 32 and abs(wl.tau[0] - 0.05) < 1e-15 and abs(wl.tau[-1] - 1.6) < 1e-14
    np.testing.assert_allclose(np.diff(wl.tau), 0.05, rtol=1e-12)
    np.testing.assert_allclose(wl.sigma, 1e-4 * wl.F_true, rtol=1e-15)
    z = (wl.Ft - wl.F_true) / wl.sigma
    assert abs(z.mean()) < 0.6 and 0.4 < z.std() < 1.6
    # truncation at omega_max = 10 removes ~2.6% of the 4.0/0.5 peak (A21)
    assert abs(W.lorentzian_mass(4.0, 0.5, 10.0, np.inf) - 0.0265) < 5e-4


def test_large_family_and_quadrature():
    wl = W.large_512x128(n_sweeps=10, n_walkers=16)
    t = wl.target
    assert np.all((t.centres >= 0.5) & (t.centres <= 8.0))
    assert np.all((t.widths >= 0.05) & (t.widths <= 1.0))
    assert abs(t.weights.sum() - 1.0) < 1e-15
    assert wl.omega.size == 512 and wl.tau.size == 128
    np.testing.assert_allclose(wl.F_true, _closed_F(t, wl.tau), rtol=1e-10)
    np.testing.assert_allclose(wl.sigma, 1e-5 * wl.F_true, rtol=1e-15)
    # seeded: the same data seed reproduces the same inputs
    wl2 = W.large_512x128(n_sweeps=10, n_walkers=16)
    assert np.array_equal(wl.Ft, wl2.Ft)


def test_geometric_schedule():
    T = W.geometric_schedule(1e2, 1e-3, 2000)
    assert T[0] == 1e2 and abs(T[-1] / 1e-3 - 1) < 1e-12
    np.testing.assert_allclose(T[1:] / T[:-1], (1e-5) ** (1 / 1999), rtol=1e-12)


def _closed_band_F(target, tau):
    """(1/2pi) int_lo^hi S e^{-omega tau} d omega for Lorentzians clipped to
    [lo, hi]: int_lo^hi e^{-omega tau}/(omega - z) = e^{-z tau}[E1((lo - z) tau) - E1((hi - z) tau)]."""
    tau = np.asarray(tau, dtype=np.float64)
    tot = np.zeros_like(tau)
    for c, w0, g in zip(target.weights, target.centres, target.widths):
        z = complex(w0, g)
        t = np.where(tau == 0.0, 1e-300, tau)
        val = np.exp(-z * t) * (exp1((target.lo - z) * t) - exp1((target.hi - z) * t))
        tot += c * np.imag(val) / np.pi
    tot = np.where(tau == 0.0, sum(c * W.lorentzian_mass(w0, g, target.lo, target.hi)
                                   for c, w0, g in zip(target.weights, target.centres, target.widths)), tot)
    return target.norm * tot / (2 * np.pi)


def test_paper_band_transform_and_moments():
    """Eq. lorentzian-band: the clipped band's transform against the
    exponential-integral closed form, unit zeroth moment, and (by symmetry of
    the two equal peaks about 1.5 on the symmetric band) first moment 1.5."""
    wl = W.paper_band("none")
    np.testing.assert_allclose(wl.F_true[1:], _closed_band_F(wl.target, wl.tau[1:]), rtol=1e-11)
    assert abs(wl.F_true[0] - 1.0 / (2 * np.pi)) < 1e-13
    assert abs(wl.m0 - 1.0) < 1e-12 and abs(wl.m1 - 1.5) < 1e-12
    assert wl.sigma is None and np.array_equal(wl.Ft, wl.F_true)
    assert wl.omega.size == 1000 and wl.n_walkers == 1500


def test_resampled_noise_generator():
    """Sec. 5.1 generator: the estimate is unbiased (within 5 standard errors
    at every lag), its standard error shrinks as 1/sqrt(n_seq), and at lag 0
    it matches the Gaussian closed form (Isserlis: the variance of the mean
    of x_i^2 over a sequence is 2 sum_ij C_ij^2 / L^2)."""
    tgt = W.Target([1.0, 2.0], [1.0, 1.0], [1.0, 1.0], 3.5, lo=0.5, hi=2.5)
    tau = 0.1 * np.arange(32)
    F, est, sig, m0, m1 = W.resampled_data(tgt, tau, 40000, 3)
    assert np.all(np.abs(est - F) <= 5 * sig)
    _, _, sig4, _, _ = W.resampled_data(tgt, tau, 160000, 4)
    assert np.all(np.abs(sig4 / sig - 0.5) < 0.05)
    L = 2 * tau.size
    Fl, _, _ = W.transform_quadrature(tgt, 0.1 * np.arange(L))
    C = Fl[np.abs(np.arange(L)[:, None] - np.arange(L)[None, :])]
    expect = np.sqrt(2.0 * np.sum(C * C) / L ** 2 / 160000)
    assert abs(sig4[0] / expect - 1) < 0.03


def test_band_skew_of_the_exact_band():
    """The skew of the exact band, binned: |mass(0.5, 1.5) - mass(1.5, 2.5)| /
    mass(0.5, 2.5) in closed form (zero here: the two equal peaks sit
    symmetrically about 1.5), to within the one bin split at 1.5; and 1 for
    a spectrum entirely on one side."""
    wl = W.paper_band("none")
    edges = np.linspace(0.0, 3.5, wl.omega.size + 1)
    bins = np.zeros(wl.omega.size)
    for c, w0, g in zip(wl.target.weights, wl.target.centres, wl.target.widths):
        lo, hi = np.clip(edges[:-1], 0.5, 2.5), np.clip(edges[1:], 0.5, 2.5)
        bins += c * (np.arctan((hi - w0) / g) - np.arctan((lo - w0) / g)) / np.pi
    one_bin = bins.max() / bins.sum()
    assert W.band_skew(bins, wl.omega) <= one_bin
    skewed = W.Target([1.0, 2.0], [1.0, 1.0], [2.0, 1.0], 3.5, lo=0.5, hi=2.5)
    m = [sum(c * W.lorentzian_mass(w0, g, a, b) for c, w0, g in zip(skewed.weights, skewed.centres, skewed.widths))
         for a, b in ((0.5, 1.5), (1.5, 2.5))]
    bins2 = np.zeros(wl.omega.size)
    for c, w0, g in zip(skewed.weights, skewed.centres, skewed.widths):
        lo, hi = np.clip(edges[:-1], 0.5, 2.5), np.clip(edges[1:], 0.5, 2.5)
        bins2 += c * (np.arctan((hi - w0) / g) - np.arctan((lo - w0) / g)) / np.pi
    assert abs(W.band_skew(bins2, wl.omega) - abs(m[0] - m[1]) / sum(m)) <= one_bin
    assert W.band_skew(np.where(wl.omega < 1.5, 1.0, 0.0), wl.omega) == 1.0
