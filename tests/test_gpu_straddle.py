"""Long steps that cross span boundaries (L divides the map period, not the
spans) through the C ABI against the FP64 oracle: full window with a node on
the boundary, blocked with the boundary between nodes, both schedules, the
reverse pass refusing such plans, and a batch whose long steps cross them."""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import TOL_F32, TOL_F64, rel_l2, say, to_dev, to_host
from workloads import WORKLOADS, Grid, dm_map, wdm_field

pytestmark = pytest.mark.gpu

TOL = {0: TOL_F32, 1: TOL_F64}


@pytest.mark.parametrize("prec", [1, 0])
def test_full_window_steps_across_boundaries(prec):
    """L = 1/7, M = 6: the step [3/7, 4/7] crosses z = 0.5 with its node 3 on it."""
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    dmm = w.dmmap.__class__(**{**w.dmmap.__dict__, "sigma": (1.0, 2.0)})
    a = w.field()
    L = 1.0 / 7.0
    say("straddle full window", prec)
    plan = P.MPAPlan(w.grid.n, w.grid.dt, dmm, L, 6, 3, 0, 0, prec)
    x = to_dev(a, prec)
    plan.propagate(x, 0.0, 2.0)
    ref = O.mpa_propagate(a, w.grid.dt, dmm, L, 6, 3, 0.0, 2.0)
    assert rel_l2(to_host(x), ref) < TOL[prec]


@pytest.mark.parametrize("prec,schedule", [(1, 0), (0, 0), (0, 1)])
def test_blocked_steps_across_boundaries(prec, schedule):
    import paper_1101_0086_amd as P
    n, dt, B = 1 << 13, 10.0 / 1024, 1024
    a = wdm_field(Grid(n, dt), 64, 4, "ook", np.random.default_rng(33))
    band = 65.0
    halo = B // 8
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(1.0 / (0.25 * halo * dt / rate))
    k += 1 - k % 2                                   # odd: L divides the period, not the spans
    L = 1.0 / k
    dmm = dm_map(beta3=0.1)
    m0 = k // 2 - 2
    z0, z1 = m0 * L, (m0 + 5) * L
    say("straddle blocked", prec, schedule)
    plan = P.MPAPlan(n, dt, dmm, L, 3, 2, B, halo, prec, band, schedule=schedule)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    ref = O.mpa_propagate(a, dt, dmm, L, 3, 2, z0, z1, B, halo)
    assert rel_l2(to_host(x), ref) < TOL[prec]


def test_reverse_pass_refuses_boundary_crossing_plans():
    import torch
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    plan = P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, 1.0 / 7.0, 6, 2, 0, 0, 1)
    x = to_dev(w.field(), 1)
    ck = plan.propagate_checkpointed(x, 0.0, 1.0)
    with pytest.raises(P.MPAError) as e:
        plan.adjoint(ck, torch.zeros_like(x), 0.0, 1.0)
    assert e.value.status == P._lib.MPA_EUNSUPPORTED


def test_batch_steps_across_boundaries():
    """A batch (two instances, sigma scales 1 and 1.5, span sigmas 1 and 2)
    whose long steps cross span boundaries: each instance against the
    oracle run with its own sigma (the map's times its scale), FP64."""
    import paper_1101_0086_amd as P
    dt, B = 10.0 / 1024, 1024
    ns, scales = [8192, 4096], [1.0, 1.5]
    fields = [wdm_field(Grid(n, dt), n // 128, 4, "ook", np.random.default_rng(40 + i)) for i, n in enumerate(ns)]
    band = 65.0
    halo = B // 8
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(1.0 / (0.25 * halo * dt / rate))
    k += 1 - k % 2                                   # odd: L divides the period, not the spans
    L = 1.0 / k
    base = dm_map(beta3=0.1)
    dmm = base.__class__(**{**base.__dict__, "sigma": (1.0, 2.0)})
    m0 = k // 2 - 2
    z0, z1 = m0 * L, (m0 + 5) * L
    say("straddle batch")
    bp = P.MPABatchPlan(ns, dt, dmm, L, 3, 2, B, halo, P.MPA_C128, band, sigma_scale=scales)
    x = to_dev(np.concatenate(fields), 1)
    bp.propagate(x, z0, z1)
    got = [to_host(v) for v in bp.split(x)]
    bp.close()
    for a, sc, g in zip(fields, scales, got):
        di = dmm.__class__(**{**dmm.__dict__, "sigma": tuple(sc * s for s in dmm.sigma)})
        ref = O.mpa_propagate(a, dt, di, L, 3, 2, z0, z1, B, halo)
        assert rel_l2(g, ref) < TOL_F64, sc
