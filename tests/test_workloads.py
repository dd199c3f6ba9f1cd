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
