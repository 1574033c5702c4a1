"""Oracle pins from the paper's accuracy analysis (Eqs. 5 and 7).

* The MPA error is twice the split-step error at equal M (the value printed
  in the text, read from tests/golden/paper_numbers.json), independent of n
  for n >= 3.
* The absolute leading terms converge, as L -> 0, to the printed P_L:
  MPA error -> i (L^3 / M^2) sigma P_L (Eq. 7 as printed) and split-step
  error -> -i (L^3 / (2 M^2)) sigma P_L.  Two readings are needed and are
  recorded in the design notes: "L-hat A0-bar" is the complex conjugate of
  L-hat applied to A0, and Eq. 5 carries the opposite sign (the split-step
  is a midpoint rule and the MPA a trapezoid rule for the same first-order
  Duhamel integral, so their errors have opposite signs).
* The iteration floor: at fixed M the distance between the n-th sweep and
  the converged sweep shrinks by a factor of order L / z_nl per sweep.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def _weak_pulse(n, T, carrier, amp):
    dt = T / n
    t = dt * np.arange(n) - T / 2
    return dt, amp * np.exp(-t * t / 2) * np.exp(-1j * carrier * t)


def _ss_reference(a0, omega, b2, b3, sig, gam, L, m_fine):
    r1 = O.ss_long_step(a0, omega, b2, b3, sig, gam, L, m_fine)
    r2 = O.ss_long_step(a0, omega, b2, b3, sig, gam, L, 2 * m_fine)
    return (4 * r2 - r1) / 3


def test_mpa_error_is_twice_split_step_error():
    gold = json.load(open(GOLDEN))["mpa_over_ss_error_ratio"]["value"]
    n, T = 1024, 64.0
    dt, a0 = _weak_pulse(n, T, 3.0, 0.1)        # z_nl = 100 z_disp, L = z_disp
    omega = O.omega_grid(n, dt)
    b2, b3, sig, gam, L = 1.0, 0.1, 1.0, 0.0, 1.0
    ref = _ss_reference(a0, omega, b2, b3, sig, gam, L, 4096)
    for M in (16, 32, 64):
        e_ss = O.rel_l2(O.ss_long_step(a0, omega, b2, b3, sig, gam, L, M), ref)
        ratios = [O.rel_l2(O.mpa_long_step(a0, omega, b2, b3, sig, gam, L, M, nit), ref) / e_ss
                  for nit in (3, 4, 5)]
        for r in ratios:
            assert abs(r - gold) < 0.05 * gold
        assert max(ratios) - min(ratios) < 0.01     # n >= 3: independent of n


def _p_l(a, omega, b2, b3, gam):
    """P_L as printed after Eq. 5, with L-hat the linear operator of Eq. 1
    (Fourier symbol beta2 omega^2/2 + beta3 omega^3/6 + i gamma) and
    "L-hat A-bar" read as conj(L-hat A)."""
    sym = 0.5 * b2 * omega ** 2 + b3 * omega ** 3 / 6 + 1j * gam

    def lop(f):
        return O.paper_ifft(sym * O.paper_fft(f))

    la = lop(a)
    ab = np.conj(a)
    p = np.abs(a) ** 2
    return ((1 / 6) * ab * la ** 2 - (1 / 3) * a * np.abs(la) ** 2
            + (1 / 6) * p * lop(la) - (1 / 3) * lop(p * la)
            + (1 / 12) * a ** 2 * np.conj(lop(la)) + (1 / 6) * lop(a ** 2 * np.conj(la))
            + (1 / 12) * lop(lop(p * a)))


def test_leading_error_terms_match_printed_p_l():
    n, T = 512, 48.0
    dt, a0 = _weak_pulse(n, T, 1.0, 0.1)
    omega = O.omega_grid(n, dt)
    b2, b3, sig, gam, M = 1.0, 0.3, 1.0, 0.05, 4
    pl = _p_l(a0, omega, b2, b3, gam)
    dev_ss, dev_mpa = [], []
    for L in (0.02, 0.01, 0.005):
        ref = _ss_reference(a0, omega, b2, b3, sig, gam, L, 1024)
        e_ss = ref - O.ss_long_step(a0, omega, b2, b3, sig, gam, L, M)
        e_mpa = ref - O.mpa_long_step(a0, omega, b2, b3, sig, gam, L, M, 4)
        lead = 1j * L ** 3 / M ** 2 * sig * pl
        dev_ss.append(O.rel_l2(e_ss, -0.5 * lead))
        dev_mpa.append(O.rel_l2(e_mpa, lead))
    # the relative deviation is the next order, O(L): it halves with L
    for dev in (dev_ss, dev_mpa):
        assert dev[-1] < 0.08
        assert 1.8 < dev[0] / dev[1] < 2.2 and 1.8 < dev[1] / dev[2] < 2.2


def test_iteration_floor_shrinks_by_l_over_znl_per_sweep():
    n, T = 512, 48.0
    L = 0.5
    for amp2, tol in ((0.05, 0.0), (0.2, 0.0)):
        dt, a0 = _weak_pulse(n, T, 2.0, math.sqrt(amp2))
        omega = O.omega_grid(n, dt)
        args = (omega, 1.0, 0.1, 1.0, 0.0, L, 64)
        _, its = O.mpa_long_step(a0, *args, 12, return_iterates=True)
        conv = its[-1]
        err = [O.rel_l2(x, conv) for x in its[1:6]]
        rate = L * amp2                      # L / z_nl with z_nl = 1 / (sigma p^2)
        for e0, e1 in zip(err, err[1:]):
            assert 0.05 * rate < e1 / e0 < 1.0 * rate
