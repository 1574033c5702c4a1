"""GPU parity of the split-step comparator (Eq. 4) against the oracle."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_util import TOL_F32, TOL_F64, rel_l2, say, to_dev, to_host
from workloads import WORKLOADS

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [1, 0])
def test_split_step_one_period(prec):
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    a = w.field()
    dz = 0.05 / 8
    say("ss one period", prec)
    plan = P.SSPlan(w.grid.n, w.grid.dt, w.dmmap, dz, prec)
    x = to_dev(a, prec)
    plan.propagate(x, 0.0, 1.0)
    got = to_host(x)
    plan.close()
    ref = O.ss_propagate(a, w.grid.dt, w.dmmap, dz, 0.0, 1.0)
    assert rel_l2(got, ref) < (TOL_F64 if prec == 1 else TOL_F32)


def test_split_step_partial_runs():
    """Start and end inside spans: runs split at the span change and amplifier."""
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    a = w.field()
    dz = 0.05 / 4
    say("ss partial runs")
    plan = P.SSPlan(w.grid.n, w.grid.dt, w.dmmap, dz, 1)
    x = to_dev(a, 1)
    plan.propagate(x, 0.3, 1.2)
    got = to_host(x)
    plan.close()
    ref = O.ss_propagate(a, w.grid.dt, w.dmmap, dz, 0.3, 1.2)
    assert rel_l2(got, ref) < TOL_F64


@pytest.mark.parametrize("n,prec", [(1 << 13, 1), (1 << 14, 0), (1 << 15, 1), (1 << 18, 0), (1 << 20, 1),
                                    (1 << 22, 0)])
def test_split_step_four_step_path(n, prec):
    """Windows above one workgroup: row/column kernels of the four-step FFT,
    across the span change at z = 0.5, against the oracle's Eq. 4."""
    import paper_1101_0086_amd as P
    from workloads import Grid, dm_map
    from workloads.wdm import _fast_wdm_field
    dt = 10.0 / 1024
    a = _fast_wdm_field(Grid(n, dt), n // 1024, 8, "ook", np.random.default_rng(9))
    dmm = dm_map(beta3=0.1)
    dz = 0.5 / 4000
    z0, z1 = 0.5 - 4 * dz, 0.5 + 4 * dz
    say("ss four-step", n, prec)
    plan = P.SSPlan(n, dt, dmm, dz, prec)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    got = to_host(x)
    plan.close()
    ref = O.ss_propagate(a, dt, dmm, dz, z0, z1)
    assert rel_l2(got, ref) < (TOL_F64 if prec == 1 else TOL_F32)


def test_stateless_split_step_equals_the_plan():
    """ss_propagate (no plan) gives bitwise the field of ss_plan_propagate."""
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    a = w.field()
    dz = 0.05 / 8
    say("ss stateless")
    plan = P.SSPlan(w.grid.n, w.grid.dt, w.dmmap, dz, 1)
    x = to_dev(a, 1)
    plan.propagate(x, 0.0, 1.0)
    plan.close()
    y = P.ss_propagate(to_dev(a, 1), w.grid.dt, w.dmmap, dz, 0.0, 1.0)
    assert np.array_equal(to_host(x), to_host(y))
