"""Node-parallel schedule (the paper's sweep-by-sweep order, every node of a
sweep its own workgroup) through the C ABI, against the fused wavefront
kernel, whose operations and sums it repeats in the same order, and the FP64
oracle.  FP32 plans give bitwise the wavefront's field.  FP64 plans agree
with it to the last bits (max relative difference of order 1e-16: the
compiler fuses a few FP64 products into additions differently in the two
kernels; with implicit fusion switched off they are bitwise equal too, at a
3-6 % cost in speed)."""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import centred_shift, TOL_F32, TOL_F64, rel_l2, say, to_dev, to_host
from workloads import WORKLOADS, Grid, dm_map, wdm_field

pytestmark = pytest.mark.gpu

TOL = {0: TOL_F32, 1: TOL_F64}


def _same(wf, npl, prec):
    if prec == 0:
        assert np.array_equal(wf, npl)
    else:
        assert np.abs(wf - npl).max() <= 1e-14 * np.abs(wf).max()


def _run(a, grid, dmmap, L, M, nit, block, halo, prec, z0, z1, band, schedule, shift=0):
    import paper_1101_0086_amd as P
    plan = P.MPAPlan(grid.n, grid.dt, dmmap, L, M, nit, block, halo, prec, band, schedule=schedule, shift=shift)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    out = to_host(x)
    plan.close()
    return out


def _blocked(block, n=1 << 14, ch=8, seed=21):
    dt = 10.0 / 1024
    grid = Grid(n, dt)
    a = wdm_field(grid, n // 1024 * 8, ch, "ook", np.random.default_rng(seed))
    band = 0.5 * (ch - 1) * 40 + 5
    halo = block // 8
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(0.5 / (0.25 * halo * dt / rate))
    while (0.5 / k) * rate > 0.25 * halo * dt:
        k += 1
    return grid, a, band, halo, 0.5 / k


@pytest.mark.parametrize("block,M,nit,prec", [(512, 1, 1, 0), (1024, 3, 2, 1), (2048, 2, 3, 0),
                                              (4096, 4, 2, 0), (4096, 4, 2, 1), (4096, 5, 1, 0)])
def test_bitwise_equal_to_wavefront_and_close_to_oracle(block, M, nit, prec):
    import paper_1101_0086_amd as P
    grid, a, band, halo, L = _blocked(block)
    dmmap = dm_map(beta3=0.1)
    z0, z1 = 0.5 - 2 * L, 0.5 + 2 * L                  # across the span change
    say("node-parallel", block, M, nit, prec)
    wf = _run(a, grid, dmmap, L, M, nit, block, halo, prec, z0, z1, band, P.MPA_WAVEFRONT)
    npl = _run(a, grid, dmmap, L, M, nit, block, halo, prec, z0, z1, band, P.MPA_NODE_PARALLEL)
    _same(wf, npl, prec)
    ref = O.mpa_propagate(a, grid.dt, dmmap, L, M, nit, z0, z1, block, halo)
    assert rel_l2(npl, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
def test_shifted_windows(prec):
    """Windows shifted against their cores: the node-parallel schedule's
    gather and scatter follow the same shift."""
    import paper_1101_0086_amd as P
    grid, a, band, halo, L = _blocked(2048)
    dmmap = dm_map(beta3=0.1)
    sh = centred_shift(band, dmmap, L, grid.dt, halo)   # middle of the band's group delay over L
    z0, z1 = 0.5 - 2 * L, 0.5 + 2 * L
    say("node-parallel shifted", prec, sh)
    wf = _run(a, grid, dmmap, L, 2, 2, 2048, halo, prec, z0, z1, band, P.MPA_WAVEFRONT, sh)
    npl = _run(a, grid, dmmap, L, 2, 2, 2048, halo, prec, z0, z1, band, P.MPA_NODE_PARALLEL, sh)
    _same(wf, npl, prec)
    ref = O.mpa_propagate(a, grid.dt, dmmap, L, 2, 2, z0, z1, 2048, halo, sh)
    assert rel_l2(npl, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
def test_full_window_small_workload(prec):
    """4096 modes, one full window, M = 16 nodes (16 node workgroups per
    sweep), 3 sweeps, one DM period across the span change and amplifier."""
    import paper_1101_0086_amd as P
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    a = w.field()
    say("node-parallel full window", prec)
    npl = _run(a, w.grid, w.dmmap, s.L, s.M, s.n_iter, 0, 0, prec, 0.0, 1.0, 0.0, P.MPA_NODE_PARALLEL)
    wf = _run(a, w.grid, w.dmmap, s.L, s.M, s.n_iter, 0, 0, prec, 0.0, 1.0, 0.0, P.MPA_WAVEFRONT)
    _same(wf, npl, prec)
    ref = O.mpa_propagate(a, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, 0.0, 1.0)
    assert rel_l2(npl, ref) < TOL[prec]


def test_bench_configuration_bitwise():
    """The 2^18-mode 8-channel workload in the benchmark's launch
    configuration (86 blocks x 4 nodes per sweep), 40 long steps."""
    import paper_1101_0086_amd as P
    w = WORKLOADS["wdm8_n262144_f32"]
    s = w.mpa
    a = w.field()
    say("node-parallel bench configuration")
    z1 = 40 * s.L
    wf = _run(a, w.grid, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, 0, 0.0, z1, s.omega_band, P.MPA_WAVEFRONT)
    npl = _run(a, w.grid, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, 0, 0.0, z1, s.omega_band,
               P.MPA_NODE_PARALLEL)
    assert np.array_equal(wf, npl)


def test_adjoint_of_a_node_parallel_plan():
    """The reverse pass recomputes each long step with the fused kernel; for a
    node-parallel plan its checkpoints come from the node-parallel forward,
    which is bitwise the same, so the gradients agree bitwise too."""
    import paper_1101_0086_amd as P
    grid, a, band, halo, L = _blocked(1024)
    dmmap = dm_map(beta3=0.1)
    g0 = np.random.default_rng(22).normal(size=a.size) + 0j
    res = []
    for sched in (P.MPA_WAVEFRONT, P.MPA_NODE_PARALLEL):
        plan = P.MPAPlan(grid.n, grid.dt, dmmap, L, 2, 2, 1024, halo, 0, band, schedule=sched)
        x = to_dev(a, 0)
        z0, z1 = 1.0 - 3 * L, 1.0 + 3 * L           # across an amplifier and a period start
        ck = plan.propagate_checkpointed(x, z0, z1)
        g = to_dev(g0, 0)
        pg = plan.adjoint(ck, g, z0, z1)
        res.append((to_host(x), to_host(g), pg.cpu().numpy()))
        plan.close()
    for u, v in zip(res[0], res[1]):
        assert np.array_equal(u, v)
