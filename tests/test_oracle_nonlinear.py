"""Oracle pins: the nonlinear term, the Picard/trapezoid machinery of Eq. 6
and the split-step of Eq. 4.

With beta2 = beta3 = 0 the problem is pointwise in t and Eq. 6 reduces to a
scalar recursion in phi = sigma |a|^2 dz, whose iterates have closed forms
derived by hand here (not by re-running the recursion):

* one sweep: psi^(1)_M = psi_0 (1 + i Phi), Phi = sigma |a|^2 L (Euler over L);
* two sweeps: psi^(2)_M / psi_0 = 1 + i Phi - Phi^2/2 + i Phi^3 (1/3 + 1/(6 M^2))
  - Phi^4 (1/4 + 1/(4 M^2)), from the trapezoid sums of j, j^2, j^3;
* n -> infinity: the implicit trapezoid (Cayley) rotation
  psi_0 ((1 + i phi/2) / (1 - i phi/2))^M.

Further: SPM with loss and the fundamental soliton are reached at second
order in dz by both methods; split-step conserves energy and is time
reversible; the MPA with many sweeps equals the sequential implicit
trapezoid rule applied to Eq. 2.
"""
import math

import numpy as np
import pytest

import oracle as O


def _pointwise_setup(n=64, seed=5):
    rng = np.random.default_rng(seed)
    a0 = 0.6 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    omega = O.omega_grid(n, 0.1)
    return a0, omega


def test_first_sweep_is_euler_over_the_long_step():
    a0, omega = _pointwise_setup()
    sigma, L, M = 0.8, 0.3, 6
    out = O.mpa_long_step(a0, omega, 0.0, 0.0, sigma, 0.0, L, M, 1)
    expect = a0 * (1 + 1j * sigma * np.abs(a0) ** 2 * L)
    assert np.max(np.abs(out - expect)) < 1e-14


@pytest.mark.parametrize("M", [1, 2, 5, 9])
def test_second_sweep_closed_form(M):
    a0, omega = _pointwise_setup()
    sigma, L = 0.8, 0.3
    out = O.mpa_long_step(a0, omega, 0.0, 0.0, sigma, 0.0, L, M, 2)
    ph = sigma * np.abs(a0) ** 2 * L
    m2 = 1.0 / (M * M)
    factor = (1 + 1j * ph - ph ** 2 / 2 + 1j * ph ** 3 * (1 / 3 + m2 / 6)
              - ph ** 4 * (1 / 4 + m2 / 4))
    assert np.max(np.abs(out - a0 * factor)) < 1e-14


def test_many_sweeps_converge_to_cayley_rotation():
    a0, omega = _pointwise_setup()
    sigma, L, M = 0.8, 0.3, 7
    out = O.mpa_long_step(a0, omega, 0.0, 0.0, sigma, 0.0, L, M, 80)
    phi = sigma * np.abs(a0) ** 2 * L / M
    expect = a0 * ((1 + 0.5j * phi) / (1 - 0.5j * phi)) ** M
    assert np.max(np.abs(out - expect)) < 1e-14


def test_many_sweeps_equal_sequential_implicit_trapezoid():
    n, T = 256, 40.0
    dt = T / n
    t = dt * np.arange(n) - T / 2
    a0 = 0.4 * np.exp(-t * t / 2) * np.exp(-2j * t)
    omega = O.omega_grid(n, dt)
    args = (omega, 1.0, 0.2, 1.0, 0.03, 0.5, 10)
    x = O.mpa_long_step(a0, *args, 60)
    y = O.if_trapezoid_long_step(a0, *args)
    assert O.rel_l2(x, y) < 1e-14


def _spm_loss_exact(a0, sigma, gamma, z):
    """beta = 0 in Eq. 1 with G = -gamma: |A| = |A0| e^{-gamma z} and the phase
    grows by sigma |A0|^2 (1 - e^{-2 gamma z}) / (2 gamma)."""
    return a0 * math.exp(-gamma * z) * np.exp(
        1j * sigma * np.abs(a0) ** 2 * (1 - math.exp(-2 * gamma * z)) / (2 * gamma))


def test_spm_with_loss_second_order_both_methods():
    a0, omega = _pointwise_setup(seed=9)
    a0 = a0 * (0.25 / 0.6)          # keep sigma |a|^2 L small: Picard over L contracts
    sigma, gamma, L = 1.0, 0.4, 0.8
    exact = _spm_loss_exact(a0, sigma, gamma, L)
    e_ss = [O.rel_l2(O.ss_long_step(a0, omega, 0, 0, sigma, gamma, L, M), exact)
            for M in (16, 32, 64)]
    e_mpa = [O.rel_l2(O.mpa_long_step(a0, omega, 0, 0, sigma, gamma, L, M, 40), exact)
             for M in (16, 32, 64)]
    for e in (e_ss, e_mpa):
        assert 3.8 < e[0] / e[1] < 4.2 and 3.8 < e[1] / e[2] < 4.2


def _soliton(t, z):
    """beta2 = -1, sigma = 1, no loss: A = sech(t) e^{i z / 2} solves Eq. 1
    (sech'' = sech - 2 sech^3)."""
    return np.exp(0.5j * z) / np.cosh(t)


def test_fundamental_soliton_both_methods():
    n, T = 1024, 64.0
    dt = T / n
    t = dt * np.arange(n) - T / 2
    a0 = _soliton(t, 0.0)
    omega = O.omega_grid(n, dt)
    Z = 2.0
    exact = _soliton(t, Z)
    e_ss, e_mpa = [], []
    for steps in (40, 80):
        e_ss.append(O.rel_l2(O.ss_long_step(a0, omega, -1.0, 0, 1.0, 0, Z, steps), exact))
        # long steps of 0.05 with 5 sweeps; M nodes per long step
        out = a0
        L = 0.05
        for _ in range(int(round(Z / L))):
            out = O.mpa_long_step(out, omega, -1.0, 0, 1.0, 0, L, steps // 40, 5)
        e_mpa.append(O.rel_l2(out, exact))
    assert e_ss[1] < 2e-4 and 3.6 < e_ss[0] / e_ss[1] < 4.4
    assert e_mpa[1] < 5e-4 and 3.3 < e_mpa[0] / e_mpa[1] < 4.4


def test_split_step_energy_and_reversibility():
    rng = np.random.default_rng(11)
    n, dt = 512, 0.05
    a0 = 0.5 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    omega = O.omega_grid(n, dt)
    out = O.ss_long_step(a0, omega, 2.0, 0.5, 1.3, 0.0, 0.7, 13)
    assert abs(np.sum(np.abs(out) ** 2) / np.sum(np.abs(a0) ** 2) - 1) < 1e-13
    back = O.ss_long_step(out, omega, -2.0, -0.5, -1.3, 0.0, 0.7, 13)
    assert O.rel_l2(back, a0) < 1e-13


def test_mpa_energy_drift_vanishes_at_second_order():
    n, T = 512, 40.0
    dt = T / n
    t = dt * np.arange(n) - T / 2
    a0 = 0.5 * np.exp(-t * t / 2) * (1 + 0.5 * np.exp(-3j * t))
    omega = O.omega_grid(n, dt)
    e0 = np.sum(np.abs(a0) ** 2)
    drift = []
    for M in (8, 16, 32):
        out = O.mpa_long_step(a0, omega, 1.0, 0.1, 1.0, 0.0, 0.5, M, 6)
        drift.append(abs(np.sum(np.abs(out) ** 2) / e0 - 1))
    assert drift[0] > 1e-12
    assert 3.5 < drift[0] / drift[1] < 4.5 and 3.5 < drift[1] / drift[2] < 4.5
