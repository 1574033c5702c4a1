"""Distributed gain in G(z) (Eq. 1 allows any G): the oracle's integral of G,
its use in the MPA long step, and the lumped-gain rule, pinned by numerical
quadrature of the definition, the exact linear solution, transparency over
an amplifier period and the NLSE energy balance d/dz int |A|^2 = 2 G int |A|^2;
the split-step with distributed gain, pinned the same way."""
import math

import numpy as np
from scipy.integrate import quad

import oracle as O
from workloads import Grid, dm_map, wdm_field
from workloads.wdm import DMMap


def _map(g0=0.2, alpha=3.0, gamma=0.05, beta3=0.1, sigma=1.0):
    m = dm_map(beta3=beta3, sigma=sigma, gamma=gamma)
    return DMMap(**{**m.__dict__, "raman_g0": g0, "raman_alpha": alpha})


def _G(dmm, zeta):
    return -dmm.gamma + dmm.raman_g0 * math.exp(-dmm.raman_alpha * (dmm.z_amp - zeta))


def test_gain_integral_matches_quadrature():
    dmm = _map()
    for zeta0, h in ((0.0, 0.3), (0.25, 0.5), (0.9, 0.1), (0.5, 0.0)):
        ref = quad(lambda z: _G(dmm, z), zeta0, zeta0 + h, epsabs=1e-14, epsrel=1e-14)[0]
        assert abs(float(O.nlse.gain_integral(dmm, zeta0, h)) - ref) < 1e-13
    # transparency: one amplifier period of loss and distributed gain, then the lumped gain
    total = quad(lambda z: _G(dmm, z), 0.0, dmm.z_amp, epsabs=1e-14, epsrel=1e-14)[0]
    assert abs(math.log(O.nlse.lumped_gain(dmm)) + total) < 1e-13
    # without distributed gain the rule is the plain exp(gamma z_a)
    assert O.nlse.lumped_gain(dm_map()) == math.exp(0.05)


def test_linear_propagation_with_distributed_gain_is_exact():
    """sigma = 0: the MPA is exact; A(z1) = F^-1[F[A] e^{i beta (z1 - z0) + int G}],
    with the span phases and the quadrature integral of G, lumped gain at 1."""
    dmm = _map(sigma=0.0)
    dmm = DMMap(**{**dmm.__dict__, "sigma": (0.0, 0.0)})
    n, dt = 512, 10 / 64
    a = wdm_field(Grid(n, dt), 8, 1, "ook", np.random.default_rng(3))
    L, z0, z1 = 0.05, 0.7, 1.3
    out = O.mpa_propagate(a, dt, dmm, L, 4, 2, z0, z1)
    omega = O.omega_grid(n, dt)
    # [0.7, 1.0) lies in span 1 (beta2 = -19.8), [1.0, 1.3) in span 0 (beta2 = +20)
    ph = O.beta_phase(omega, -19.8, 0.1, 0.3) + O.beta_phase(omega, 20.0, 0.1, 0.3)
    g = (quad(lambda z: _G(dmm, z), 0.7, 1.0, epsabs=1e-14, epsrel=1e-14)[0]
         + math.log(O.nlse.lumped_gain(dmm))
         + quad(lambda z: _G(dmm, z), 0.0, 0.3, epsabs=1e-14, epsrel=1e-14)[0])
    exact = O.paper_ifft(O.paper_fft(a) * np.exp(1j * ph + g))
    assert O.rel_l2(out, exact) < 1e-12


def test_energy_balance_with_distributed_gain():
    """sigma != 0: int |A|^2 changes only through G, by exp(2 int G).  The MPA
    keeps this to its truncation error: the error falls about fourfold when
    M doubles, and the extrapolated energy matches to far below it."""
    dmm = _map()
    n, dt = 1024, 10 / 128
    a = 0.6 * wdm_field(Grid(n, dt), 8, 2, "ook", np.random.default_rng(4))
    e0 = float(np.sum(np.abs(a) ** 2))
    L, z0, z1 = 0.05, 0.2, 0.45
    g = quad(lambda z: _G(dmm, z), z0, z1, epsabs=1e-14, epsrel=1e-14)[0]
    exact = e0 * math.exp(2 * g)
    errs = []
    for M in (2, 4):
        out = O.mpa_propagate(a, dt, dmm, L, M, 4, z0, z1)
        errs.append(float(np.sum(np.abs(out) ** 2)) / exact - 1.0)
    assert abs(errs[1]) < abs(errs[0])
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert abs((4 * errs[1] - errs[0]) / 3) < 0.05 * abs(errs[1])


def test_split_step_with_distributed_gain():
    """ss_long_step_gain, pinned three ways: (1) sigma = 0 gives the exact
    linear solution with the quadrature integral of G over the run; (2) with
    sigma != 0 the energy changes by exp(2 int G) to rounding (the SPM kick
    keeps |A| and each linear half step scales the energy by exactly its
    exp(2 int G)); (3) with no distributed gain it is the uniform-loss
    split-step of Eq. 4 (merged half steps) to rounding."""
    n, dt = 512, 10 / 64
    a = 0.6 * wdm_field(Grid(n, dt), 8, 1, "ook", np.random.default_rng(6))
    omega = O.omega_grid(n, dt)
    dz, zeta0, steps = 0.01, 0.52, 30                  # [0.52, 0.82] in span 1, one amplifier period
    lin = _map(sigma=0.0)
    out = O.ss_long_step_gain(a, omega, -19.8, 0.1, 0.0, lin, zeta0, dz, steps)
    g = quad(lambda z: _G(lin, z), zeta0, zeta0 + steps * dz, epsabs=1e-14, epsrel=1e-14)[0]
    exact = O.paper_ifft(O.paper_fft(a) * np.exp(1j * O.beta_phase(omega, -19.8, 0.1, steps * dz) + g))
    assert O.rel_l2(out, exact) < 1e-12
    dmm = _map()
    out = O.ss_long_step_gain(a, omega, -19.8, 0.1, 1.0, dmm, zeta0, dz, steps)
    ratio = float(np.sum(np.abs(out) ** 2)) / float(np.sum(np.abs(a) ** 2))
    g = quad(lambda z: _G(dmm, z), zeta0, zeta0 + steps * dz, epsabs=1e-14, epsrel=1e-14)[0]
    assert abs(ratio / math.exp(2 * g) - 1.0) < 1e-12
    flat = _map(g0=0.0)
    out = O.ss_long_step_gain(a, omega, -19.8, 0.1, 1.0, flat, zeta0, dz, steps)
    ref = O.ss_long_step(a, omega, -19.8, 0.1, 1.0, flat.gamma, steps * dz, steps)
    assert O.rel_l2(out, ref) < 1e-12
    # ss_propagate across an amplifier: the run before it, the lumped gain, the run after
    z0, z1 = 0.9, 1.2
    got = O.ss_propagate(a, dt, dmm, dz, z0, z1)
    k0 = round(z0 / dz)
    ref = O.ss_long_step_gain(a, omega, -19.8, 0.1, 1.0, dmm, z0, dz, round(0.1 / dz))
    ref = ref * O.nlse.lumped_gain(dmm)
    ref = O.ss_long_step_gain(ref, omega, 20.0, 0.1, 1.0, dmm, 0.0, dz, round(0.2 / dz))
    assert k0 == 90 and O.rel_l2(got, ref) < 1e-13
