"""Long steps that cross span boundaries (L divides the map period, not the
spans) through the C ABI against the FP64 oracle: full window with a node on
the boundary, blocked with the boundary between nodes, both schedules, a
step over three spans, and a batch whose long steps cross them; the reverse
pass of such plans (field gradient and per-span parameter derivatives)
against the oracle's gradient, single fields and a batch."""
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


def _straddle_blocked_case(n=1 << 13, B=1024, seed=33):
    dt = 10.0 / 1024
    a = wdm_field(Grid(n, dt), 64, 4, "ook", np.random.default_rng(seed))
    band = 65.0
    halo = B // 8
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(1.0 / (0.25 * halo * dt / rate))
    k += 1 - k % 2                                   # odd: L divides the period, not the spans
    return a, dt, band, halo, k


@pytest.mark.parametrize("prec", [1, 0])
def test_reverse_full_window_across_a_boundary_on_a_node(prec):
    """L = 1/7, M = 6, sigma 1 and 2: the step [3/7, 4/7] crosses z = 0.5 with
    node 3 on it; field gradient and per-span derivatives against the oracle."""
    from tests.test_gpu_adjoint import _compare, _gpu_grad, _oracle, _target
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    dmm = w.dmmap.__class__(**{**w.dmmap.__dict__, "sigma": (1.0, 2.0)})
    a = w.field()
    L, M, nit = 1.0 / 7.0, 6, 2
    z0, z1 = 2.0 / 7.0, 5.0 / 7.0
    target = _target(a, w.grid.dt, np.random.default_rng(61), 0.8, 0.05, 10.0)
    _, g_out, ref_g, ref_p = _oracle(a, w.grid.dt, dmm, L, M, nit, z0, z1, target)
    say("straddle reverse full window", prec)
    plan = P.MPAPlan(w.grid.n, w.grid.dt, dmm, L, M, nit, 0, 0, prec)
    _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, prec)
    plan.close()
    _compare(prec, got_g, got_p, ref_g, ref_p)


@pytest.mark.parametrize("prec,shifted", [(1, False), (0, False), (1, True)])
def test_reverse_blocked_across_boundaries(prec, shifted):
    """Blocked plans whose boundary at 0.5 falls between two nodes of a step
    (and the map-period boundary at 1.0 on a step edge), with and without a
    window shift (the roll-off follows the step's mean coefficients)."""
    from tests.gpu_util import centred_shift
    from tests.test_gpu_adjoint import _compare, _gpu_grad, _oracle, _target
    import paper_1101_0086_amd as P
    a, dt, band, halo, k = _straddle_blocked_case()
    L = 1.0 / k
    base = dm_map(beta3=0.1)
    dmm = base.__class__(**{**base.__dict__, "sigma": (1.0, 2.0)})
    sh = centred_shift(band, dmm, L, dt, halo) if shifted else 0
    target = _target(a, dt, np.random.default_rng(62), 0.9, 0.02, band)
    m0 = k // 2 - 2
    z0, z1 = m0 * L, (m0 + 5) * L
    _, g_out, ref_g, ref_p = _oracle(a, dt, dmm, L, 3, 2, z0, z1, target, 1024, halo, sh)
    say("straddle reverse blocked", prec, sh)
    plan = P.MPAPlan(a.size, dt, dmm, L, 3, 2, 1024, halo, prec, band, shift=sh)
    _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, prec)
    plan.close()
    _compare(prec, got_g, got_p, ref_g, ref_p)


def test_step_over_three_spans_forward_and_reverse():
    """A middle span (0.05) shorter than the long step (1/7): the step
    [3/7, 4/7] overlaps three spans; forward and reverse, FP64."""
    from tests.test_gpu_adjoint import _compare, _gpu_grad, _oracle, _target
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    dmm = dm_map(beta3=0.1, beta2=(20.0, -7.0, -19.8), seg=(0.5, 0.05, 0.45))
    dmm = dmm.__class__(**{**dmm.__dict__, "sigma": (1.0, 3.0, 2.0)})
    a = w.field()
    L, M, nit = 1.0 / 7.0, 3, 2
    z0, z1 = 2.0 / 7.0, 5.0 / 7.0
    target = _target(a, w.grid.dt, np.random.default_rng(63), 0.8, 0.05, 10.0)
    out, g_out, ref_g, ref_p = _oracle(a, w.grid.dt, dmm, L, M, nit, z0, z1, target)
    say("three spans in one step")
    plan = P.MPAPlan(w.grid.n, w.grid.dt, dmm, L, M, nit, 0, 0, 1)
    x = to_dev(a, 1)
    plan.propagate(x, z0, z1)
    assert rel_l2(to_host(x), out) < TOL_F64
    _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, 1)
    plan.close()
    _compare(1, got_g, got_p, ref_g, ref_p)


def test_batch_reverse_across_boundaries():
    """Batch (two instances, sigma scales 1 and 1.5) over steps that cross
    the span change: field gradients and the summed per-span derivatives
    against the oracle run with each instance's sigma, FP64."""
    import paper_1101_0086_amd as P
    a0, dt, band, halo, k = _straddle_blocked_case()
    ns, scales = [8192, 4096], [1.0, 1.5]
    fields = [a0, wdm_field(Grid(4096, dt), 32, 4, "ook", np.random.default_rng(41))]
    L = 1.0 / k
    base = dm_map(beta3=0.1)
    dmm = base.__class__(**{**base.__dict__, "sigma": (1.0, 2.0)})
    m0 = k // 2 - 2
    z0, z1 = m0 * L, (m0 + 5) * L
    rng = np.random.default_rng(64)
    g_out = [0.1 * (rng.normal(size=n) + 1j * rng.normal(size=n)) for n in ns]
    say("straddle reverse batch")
    bp = P.MPABatchPlan(ns, dt, dmm, L, 3, 2, 1024, halo, P.MPA_C128, band, sigma_scale=scales)
    x = to_dev(np.concatenate(fields), 1)
    ck = bp.propagate_checkpointed(x, z0, z1)
    g = to_dev(np.concatenate(g_out), 1)
    pg = bp.adjoint(ck, g, z0, z1).cpu().numpy()
    got_g = [to_host(v) for v in bp.split(g)]
    bp.close()
    ref_p = np.zeros((3, 2))
    for a, go, sc, gg in zip(fields, g_out, scales, got_g):
        di = dmm.__class__(**{**dmm.__dict__, "sigma": tuple(sc * s for s in dmm.sigma)})
        ga, gs, g2, g3 = O.mpa_propagate_vjp(a, dt, di, L, 3, 2, z0, z1, go, 1024, halo)
        assert rel_l2(gg, ga) < 1e-10
        ref_p += np.stack([sc * gs, g2, g3])
    err = np.linalg.norm(pg - ref_p) / np.linalg.norm(ref_p)
    assert err < 1e-9, (err, pg, ref_p)


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


@pytest.mark.parametrize("z_amp,prec", [(1.0, 1), (1.0, 0), (2.0, 1)])
def test_distributed_gain_with_boundary_crossing_steps(z_amp, prec):
    """Distributed gain and L = 1/7 (steps across z = 0.5 and 1.5): each such
    step takes its node sigma and the gain profile of its position in the
    amplifier period (z_amp = 2: two positions per crossing step of the
    period); forward over several amplifiers against the oracle, and the
    reverse pass against the oracle's gradient (FP64)."""
    from tests.test_gpu_adjoint import _compare, _gpu_grad, _oracle, _target
    import paper_1101_0086_amd as P
    from workloads.wdm import DMMap
    w = WORKLOADS["dm1ch_n4096_f64"]
    dmm = DMMap(**{**w.dmmap.__dict__, "sigma": (1.0, 2.0), "z_amp": z_amp, "raman_g0": 0.2,
                   "raman_alpha": 3.0})
    a = w.field()
    L, M, nit = 1.0 / 7.0, 3, 2
    z0, z1 = 2.0 / 7.0, 2.0 / 7.0 + (4.0 if z_amp == 2.0 else 2.0)
    say("distributed gain with crossing steps", z_amp, prec)
    plan = P.MPAPlan(w.grid.n, w.grid.dt, dmm, L, M, nit, 0, 0, prec)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    ref = O.mpa_propagate(a, w.grid.dt, dmm, L, M, nit, z0, z1)
    assert rel_l2(to_host(x), ref) < TOL[prec]
    if prec == 1:
        zr1 = z0 + 1.0
        target = _target(a, w.grid.dt, np.random.default_rng(65), 0.8, 0.05, 10.0)
        _, g_out, ref_g, ref_p = _oracle(a, w.grid.dt, dmm, L, M, nit, z0, zr1, target)
        _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, zr1, 1)
        _compare(1, got_g, got_p, ref_g, ref_p)
    plan.close()
