"""Oracle pins: Fourier convention and the linear part of Eq. 1.

* the transform equals a brute-force DFT with kernel exp(+i omega t);
* a Gaussian under beta2 (beta3 = 0) with loss matches the closed-form
  solution of the linear part of Eq. 1 derived in the time domain;
* the centroid of a carrier-shifted pulse under beta2 and beta3 moves by the
  amount the moment equation of Eq. 1 fixes (this catches a flipped sign of
  the odd omega^3 term, which the closed Gaussian test cannot see);
* with sigma = 0 the MPA is exact for any L, M, n (psi = const solves the
  linear problem) and split-step reduces to the same linear propagation.
"""
import math

import numpy as np
import pytest

import oracle as O


def test_paper_fft_is_the_e_plus_i_omega_t_dft():
    rng = np.random.default_rng(0)
    for n in (1, 2, 3, 8, 16):
        dt = 0.37
        a = rng.normal(size=n) + 1j * rng.normal(size=n)
        t = dt * np.arange(n)
        kk = np.array([k if k < (n + 1) // 2 else k - n for k in range(n)], float)
        omega = 2 * math.pi * kk / (n * dt)
        brute = np.array([sum(a[m] * np.exp(1j * omega[k] * t[m]) for m in range(n))
                          for k in range(n)])
        assert np.max(np.abs(O.paper_fft(a) - brute)) <= 1e-13 * max(1.0, np.max(np.abs(brute)))
        # inverse: A_n = (1/N) sum_k Ahat_k exp(-i omega_k t_n)
        back = np.array([sum(brute[k] * np.exp(-1j * omega[k] * t[m]) for k in range(n)) / n
                         for m in range(n)])
        assert np.max(np.abs(O.paper_ifft(brute) - back)) <= 1e-13 * max(1.0, np.max(np.abs(back)))
        assert np.allclose(O.omega_grid(n, dt), omega, rtol=0, atol=1e-12)


def _gaussian_closed_form(t, tau, b2_int, gamma, z):
    """Linear part of Eq. 1 with beta3 = 0: A_z = -(i/2) beta2 A_tt - gamma A.
    For A(t,0) = exp(-t^2/(2 tau^2)) the solution is
    tau / sqrt(tau^2 - i B2) exp(-t^2 / (2 (tau^2 - i B2))) e^{-gamma z},
    B2 = int beta2 dz (heat kernel with complex diffusivity -i beta2 / 2)."""
    q = tau * tau - 1j * b2_int
    return tau / np.sqrt(q) * np.exp(-t * t / (2 * q)) * math.exp(-gamma * z)


@pytest.mark.parametrize("beta2", [1.5, -2.0])
def test_gaussian_linear_closed_form_all_paths(beta2):
    n, T = 1024, 80.0
    dt = T / n
    t = dt * np.arange(n) - T / 2          # pulse centred in the window
    tau, gamma, L = 1.3, 0.1, 0.6
    a0 = np.exp(-t * t / (2 * tau * tau))
    exact = _gaussian_closed_form(t, tau, beta2 * L, gamma, L)
    omega = O.omega_grid(n, dt)
    lin = O.linear_step(a0, omega, beta2, 0.0, gamma, L)
    assert np.max(np.abs(lin - exact)) < 1e-13
    for M, nit in ((1, 1), (7, 3), (16, 5)):
        mpa = O.mpa_long_step(a0, omega, beta2, 0.0, 0.0, gamma, L, M, nit)
        assert np.max(np.abs(mpa - exact)) < 1e-13
    ss = O.ss_long_step(a0, omega, beta2, 0.0, 0.0, gamma, L, 9)
    assert np.max(np.abs(ss - exact)) < 1e-13


def _centroid(t, a):
    w = np.abs(a) ** 2
    return float(np.sum(t * w) / np.sum(w))


@pytest.mark.parametrize("carrier", [-6.0, 0.0, 4.0])
def test_centroid_drift_fixes_sign_of_beta3(carrier):
    """From Eq. 1 with sigma = 0: d<t>/dz = <beta2 omega + beta3 omega^2 / 2>,
    the average over the power spectrum.  For exp(-t^2/2tau^2) exp(-i Omega t)
    the spectrum (kernel e^{+i omega t}) is centred at +Omega with variance
    1/(2 tau^2), so <t> moves by B2 Omega + B3 (Omega^2 + 1/(2 tau^2)) / 2."""
    n, T = 4096, 200.0
    dt = T / n
    t = dt * np.arange(n) - T / 2
    tau, b2, b3, L = 1.0, 0.7, 0.9, 1.5
    dw = 2 * math.pi / T
    omega_c = dw * round(carrier / dw)
    a0 = np.exp(-t * t / (2 * tau * tau)) * np.exp(-1j * omega_c * t)
    omega = O.omega_grid(n, dt)
    out = O.mpa_long_step(a0, omega, b2, b3, 0.0, 0.0, L, 4, 2)
    drift = _centroid(t, out) - _centroid(t, a0)
    expect = b2 * L * omega_c + b3 * L * (omega_c ** 2 + 1 / (2 * tau * tau)) / 2
    assert abs(drift - expect) < 1e-9 * max(1.0, abs(expect))
    # the opposite sign of the odd term gives a different drift whenever beta3 != 0
    wrong = b2 * L * omega_c - b3 * L * (omega_c ** 2 + 1 / (2 * tau * tau)) / 2
    assert abs(drift - wrong) > 0.1


def test_mpa_sigma_zero_is_exact_linear_propagation():
    """psi = const is the exact solution of the linear problem, so with
    sigma = 0 the MPA reproduces spectral propagation for any L, M, n."""
    rng = np.random.default_rng(3)
    n, dt = 256, 0.05
    a0 = rng.normal(size=n) + 1j * rng.normal(size=n)
    omega = O.omega_grid(n, dt)
    for L in (0.01, 0.4, 3.0):
        ref = O.linear_step(a0, omega, -1.3, 0.4, 0.07, L)
        for M, nit in ((1, 1), (5, 2), (12, 4)):
            out = O.mpa_long_step(a0, omega, -1.3, 0.4, 0.0, 0.07, L, M, nit)
            assert O.rel_l2(out, ref) < 1e-13
