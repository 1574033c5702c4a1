"""Distributed gain (G = -gamma + g0 exp(-alpha (z_a - zeta)), transparent
lumped amplifiers) through the C ABI against the FP64 oracle: full window
and blocked plans, both precisions, across a span change, an amplifier and a
period start; the reverse pass against the oracle gradient; split-step plans
with the profile against the oracle's split-step; a batch with the profile."""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import TOL_F32, TOL_F64, rel_l2, say, to_dev, to_host
from workloads import WORKLOADS, Grid, dm_map, wdm_field
from workloads.wdm import DMMap

pytestmark = pytest.mark.gpu

TOL = {0: TOL_F32, 1: TOL_F64}


def _raman(m, g0=0.2, alpha=3.0):
    return DMMap(**{**m.__dict__, "raman_g0": g0, "raman_alpha": alpha})


@pytest.mark.parametrize("prec", [1, 0])
def test_full_window_with_distributed_gain(prec):
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    dmm = _raman(w.dmmap)
    a = w.field()
    say("distributed gain full window", prec)
    plan = P.MPAPlan(w.grid.n, w.grid.dt, dmm, s.L, s.M, s.n_iter, 0, 0, prec)
    x = to_dev(a, prec)
    plan.propagate(x, 0.3, 2.2)
    ref = O.mpa_propagate(a, w.grid.dt, dmm, s.L, s.M, s.n_iter, 0.3, 2.2)
    assert rel_l2(to_host(x), ref) < TOL[prec]
    # without the profile the result changes by far more than the tolerance
    plain = O.mpa_propagate(a, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, 0.3, 2.2)
    assert rel_l2(plain, ref) > 1e-2


@pytest.mark.parametrize("prec", [1, 0])
def test_blocked_with_distributed_gain(prec):
    import paper_1101_0086_amd as P
    n, dt, B = 1 << 13, 10.0 / 1024, 1024
    a = wdm_field(Grid(n, dt), 64, 4, "ook", np.random.default_rng(31))
    band = 65.0
    halo = B // 8
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(0.5 / (0.25 * halo * dt / rate))
    while (0.5 / k) * rate > 0.25 * halo * dt:
        k += 1
    L = 0.5 / k
    dmm = _raman(dm_map(beta3=0.1))
    z0, z1 = 1.0 - 3 * L, 1.0 + 2 * L
    say("distributed gain blocked", prec)
    plan = P.MPAPlan(n, dt, dmm, L, 2, 2, B, halo, prec, band)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    ref = O.mpa_propagate(a, dt, dmm, L, 2, 2, z0, z1, B, halo)
    assert rel_l2(to_host(x), ref) < TOL[prec]


def test_reverse_pass_with_distributed_gain():
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    dmm = _raman(w.dmmap)
    a = w.field()
    z0, z1 = 0.8, 1.15
    out = O.mpa_propagate(a, w.grid.dt, dmm, s.L, s.M, s.n_iter, z0, z1)
    g_out = 2 * (out - 0.5 * a)
    ref_g, gs, g2, g3 = O.mpa_propagate_vjp(a, w.grid.dt, dmm, s.L, s.M, s.n_iter, z0, z1, g_out)
    say("distributed gain reverse pass")
    plan = P.MPAPlan(w.grid.n, w.grid.dt, dmm, s.L, s.M, s.n_iter, 0, 0, 1)
    x = to_dev(a, 1)
    ck = plan.propagate_checkpointed(x, z0, z1)
    g = to_dev(g_out, 1)
    pg = plan.adjoint(ck, g, z0, z1).cpu().numpy()
    assert rel_l2(to_host(g), ref_g) < 1e-10
    ref_p = np.stack([gs, g2, g3])
    assert np.linalg.norm(pg - ref_p) < 1e-9 * np.linalg.norm(ref_p)


@pytest.mark.parametrize("n,prec", [(1 << 12, 1), (1 << 12, 0), (1 << 14, 1), (1 << 14, 0)])
def test_split_step_with_distributed_gain(n, prec):
    """Split-step plans with distributed gain (one symmetric step per launch,
    each half step scaled by exp(int G) over its interval), the one-workgroup
    and the four-step paths, across a span change, an amplifier and a period
    start, against the oracle's split-step with the same G."""
    import paper_1101_0086_amd as P
    dt = 10.0 / 1024
    a = wdm_field(Grid(n, dt), n // 128, 4, "ook", np.random.default_rng(60))
    dmm = _raman(dm_map(beta3=0.1))
    dz = 0.5 / 400
    z0, z1 = 1.0 - 6 * dz, 1.0 + 5 * dz
    say("split-step distributed gain", n, prec)
    plan = P.SSPlan(n, dt, dmm, dz, prec)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    got = to_host(x)
    plan.close()
    ref = O.ss_propagate(a, dt, dmm, dz, z0, z1)
    assert rel_l2(got, ref) < TOL[prec]
    # without the profile the result differs by far more than the tolerance
    assert rel_l2(O.ss_propagate(a, dt, dm_map(beta3=0.1), dz, z0, z1), ref) > 1e-3


def test_batch_with_distributed_gain():
    """A batch (two instances, sigma scales 1 and 0.7) with distributed gain,
    across an amplifier: each instance against the oracle with its own
    sigma, FP64."""
    import paper_1101_0086_amd as P
    dt, B = 10.0 / 1024, 1024
    ns, scales = [4096, 8192], [1.0, 0.7]
    fields = [wdm_field(Grid(n, dt), n // 128, 4, "ook", np.random.default_rng(50 + i)) for i, n in enumerate(ns)]
    band = 65.0
    halo = B // 8
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(0.5 / (0.25 * halo * dt / rate))
    while (0.5 / k) * rate > 0.25 * halo * dt:
        k += 1
    L = 0.5 / k
    dmm = _raman(dm_map(beta3=0.1))
    z0, z1 = 1.0 - 3 * L, 1.0 + 2 * L
    say("distributed gain batch")
    bp = P.MPABatchPlan(ns, dt, dmm, L, 2, 2, B, halo, P.MPA_C128, band, sigma_scale=scales)
    x = to_dev(np.concatenate(fields), 1)
    bp.propagate(x, z0, z1)
    got = [to_host(v) for v in bp.split(x)]
    bp.close()
    for a, sc, g in zip(fields, scales, got):
        ref = O.mpa_propagate(a, dt, dmm.with_sigma(sc), L, 2, 2, z0, z1, B, halo)
        assert rel_l2(g, ref) < TOL_F64, sc
