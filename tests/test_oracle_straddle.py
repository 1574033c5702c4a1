"""Long steps that cross a span boundary (coefficients varying inside a long
step): beta(omega, z_j) as the exact integral of the piecewise-constant
beta2, beta3, sigma sampled at the nodes with the mean of both spans on a
boundary node.  Pinned by the exact linear solution, second-order
convergence to a converged split-step reference when a node sits on the
boundary (a one-sided sigma there would make it first order), and the
helper's integrals against direct sums."""
import numpy as np

import oracle as O
from workloads import Grid, dm_map, wdm_field


def test_step_coefficients():
    dmm = dm_map(beta3=0.1, sigma=1.0)
    dmm = dmm.__class__(**{**dmm.__dict__, "sigma": (1.0, 3.0)})
    L, M = 1.0 / 3.0, 4
    (b2, b3), sig = O.nlse.step_coefficients(dmm, L, M, 1)          # [1/3, 2/3] crosses 0.5
    zj = 1.0 / 3.0 + (L / M) * np.arange(M + 1)
    want = np.where(zj <= 0.5, 20.0 * (zj - 1 / 3), 20.0 * (0.5 - 1 / 3) - 19.8 * (zj - 0.5))
    assert np.allclose(b2, want, rtol=0, atol=1e-14)
    assert np.allclose(b3, 0.1 * (zj - 1 / 3), rtol=0, atol=1e-15)
    assert np.array_equal(sig, [1.0, 1.0, 2.0, 3.0, 3.0])         # node 2 is on the boundary
    assert O.nlse.long_step_spans(dmm, L, 1) == [0, 1]
    assert O.nlse.long_step_spans(dmm, L, 0) == [0] and O.nlse.long_step_spans(dmm, L, 2) == [1]
    # the last step of a period ends on the period boundary: one span only
    assert O.nlse.long_step_spans(dmm, 0.25, 3) == [1]


def test_linear_steps_across_boundaries_are_exact():
    dmm = dm_map(beta3=0.1, sigma=0.0)
    n, dt = 512, 10 / 64
    a = wdm_field(Grid(n, dt), 8, 1, "ook", np.random.default_rng(5))
    L = 1.0 / 3.0
    out = O.mpa_propagate(a, dt, dmm, L, 3, 2, 0.0, 1.0)            # steps 2 of 3 crosses 0.5
    ref = O.ss_propagate(a, dt, dmm, 0.5, 0.0, 1.0)                  # sigma = 0: exact too
    assert O.rel_l2(out, ref) < 1e-12


def test_second_order_with_a_node_on_the_boundary():
    dmm = dm_map(beta3=0.1, sigma=1.0, gamma=0.0, z_amp=0.0)
    dmm = dmm.__class__(**{**dmm.__dict__, "sigma": (1.0, 3.0)})
    n, dt = 256, 10 / 32
    a = 0.5 * wdm_field(Grid(n, dt), 8, 1, "ook", np.random.default_rng(6))
    L = 1.0 / 3.0
    ref, est = O.reference_propagate(a, dt, dmm, 1 / 3, 2 / 3, 64, rtol=1e-11)
    assert est < 1e-10
    errs = [O.rel_l2(O.mpa_propagate(a, dt, dmm, L, M, 4, 1 / 3, 2 / 3), ref) for M in (4, 8, 16)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs
