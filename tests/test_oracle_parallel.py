"""The CPU baseline's parallel decomposition (nodes of a sweep over threads,
the trapezoid by harmonic ranges) equals the oracle's long step."""
import numpy as np

import oracle as O
from oracle.parallel import mpa_long_step_parallel
from workloads import Grid, wdm_field


def test_parallel_decomposition_equals_the_long_step():
    n, dt = 1 << 12, 10 / 256
    a = wdm_field(Grid(n, dt), 16, 2, "ook", np.random.default_rng(3))
    om = O.omega_grid(n, dt)
    for M, nit, workers in ((4, 2, 3), (7, 3, 8), (1, 1, 2)):
        ref = O.mpa_long_step(a, om, 20.0, 0.1, 1.0, 0.05, 0.05, M, nit)
        got = mpa_long_step_parallel(a, om, 20.0, 0.1, 1.0, 0.05, 0.05, M, nit, workers=workers)
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)), (M, nit)
