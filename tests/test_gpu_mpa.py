"""GPU parity of the HIP MPA path against the FP64 oracle (through the C ABI).

Cases span several blocks with a ragged last core, every compiled block
size, 1..5 Picard sweeps, both precisions, marching across a span boundary
and an amplifier, the small full-window workload (4096 modes, FP64, ten DM
periods) and, at the full 2^18-mode 8-channel size in the launch
configuration the benchmark times, and at the largest size a plan accepts
(2^30 modes), sampled blocks that the oracle computes one at a time.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import TOL_F32, TOL_F64, rel_l2, say, to_dev, to_host
from workloads import WORKLOADS, Grid, dm_map, wdm_field

pytestmark = pytest.mark.gpu

TOL = {0: TOL_F32, 1: TOL_F64}


def _plan(w_or_grid, dmmap, L, M, nit, block, halo, prec, omega_band=0.0, shift=0):
    import paper_1101_0086_amd as P
    g = w_or_grid
    return P.MPAPlan(g.n, g.dt, dmmap, L, M, nit, block, halo, prec, omega_band, shift=shift)


def _run_mpa(a, grid, dmmap, L, M, nit, block, halo, prec, z0, z1, omega_band=0.0, shift=0):
    plan = _plan(grid, dmmap, L, M, nit, block, halo, prec, omega_band, shift)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    out = to_host(x)
    plan.close()
    return out


@pytest.mark.parametrize("prec", [1, 0])
def test_full_window_one_long_step(prec):
    w = WORKLOADS["dm1ch_n4096_f64"]
    a = w.field()
    s = w.mpa
    say("full window one long step", prec)
    got = _run_mpa(a, w.grid, w.dmmap, s.L, s.M, s.n_iter, 0, 0, prec, 0.0, s.L)
    ref = O.mpa_propagate(a, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, 0.0, s.L)
    assert rel_l2(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
def test_small_workload_ten_periods(prec):
    """4096 modes, single OOK channel, L = 0.05, M = 16, 3 sweeps: 200 long
    steps across 20 span changes and 10 amplifiers."""
    w = WORKLOADS["dm1ch_n4096_f64"]
    a = w.field()
    s = w.mpa
    z1 = float(w.periods)
    say("small workload ten periods", prec)
    got = _run_mpa(a, w.grid, w.dmmap, s.L, s.M, s.n_iter, 0, 0, prec, 0.0, z1)
    ref = O.mpa_propagate(a, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, 0.0, z1)
    err = rel_l2(got, ref)
    assert err < TOL[prec], err


def _blocked_case(block, n=1 << 15, bits=32, ch=8, seed=3):
    dt = 10.0 / 1024
    grid = Grid(n, dt)
    a = wdm_field(grid, bits, ch, "ook", np.random.default_rng(seed))
    omega_band = 0.5 * (ch - 1) * 40 + 5
    halo = block // 8
    rate = O.halo_rate(omega_band, 20.0, 0.1)
    # largest long step dividing the 0.5 spans inside the halo rule
    lmax = 0.25 * halo * dt / rate
    k = math.ceil(0.5 / lmax)
    while (0.5 / k) * rate > 0.25 * halo * dt:
        k += 1
    return grid, a, omega_band, halo, 0.5 / k


@pytest.mark.parametrize("block", [512, 1024, 2048, 4096])
@pytest.mark.parametrize("prec", [1, 0])
def test_blocked_across_span_and_amplifier(block, prec):
    grid, a, band, halo, L = _blocked_case(block)
    dmm = dm_map(beta3=0.1)
    # two long steps before and after the span change at z = 0.5, and the same at z = 1 (amplifier)
    for z0 in (0.5 - 2 * L, 1.0 - 2 * L):
        say("blocked", block, prec, z0)
        got = _run_mpa(a, grid, dmm, L, 2, 2, block, halo, prec, z0, z0 + 4 * L, band)
        ref = O.mpa_propagate(a, grid.dt, dmm, L, 2, 2, z0, z0 + 4 * L, block, halo)
        assert rel_l2(got, ref) < TOL[prec]


def _shifted_case(block, n=1 << 15, bits=32, ch=8, seed=3):
    """As _blocked_case, with the window shifted by the middle of the band's
    group-delay range over L (beta2 = +20 and -19.8, beta3 = 0.1), which
    admits the longest L dividing the spans within the halo rule."""
    dt = 10.0 / 1024
    grid = Grid(n, dt)
    a = wdm_field(grid, bits, ch, "ook", np.random.default_rng(seed))
    band = 0.5 * (ch - 1) * 40 + 5
    halo = block // 8
    ranges = [O.group_delay_range(band, b2, 0.1) for b2 in (20.0, -19.8)]
    lo, hi = min(r[0] for r in ranges), max(r[1] for r in ranges)
    k = 1
    while True:
        L = 0.5 / k
        sh = int(round(0.5 * (lo + hi) * L / dt))
        if abs(sh) <= halo // 2 and all(O.halo_excursion(band, b2, 0.1, L, sh, dt) <= 0.25 * halo * dt
                                        for b2 in (20.0, -19.8)):
            return grid, a, band, halo, L, sh
        k += 1


@pytest.mark.parametrize("block", [1024, 4096])
@pytest.mark.parametrize("prec", [1, 0])
def test_window_shift_across_span_and_amplifier(block, prec):
    """Windows moved against their cores: the shifted partition, the shifted
    roll-off and a long step longer than the unshifted halo rule admits,
    across the span change and an amplifier; the plan's automatic choice of
    the shift equals the middle of the group-delay range over both spans."""
    import paper_1101_0086_amd as P
    grid, a, band, halo, L, sh = _shifted_case(block)
    assert sh != 0
    dmm = dm_map(beta3=0.1)
    with pytest.raises(P.MPAError):       # unshifted, the same long step breaks the halo rule
        P.validate(grid.n, grid.dt, dmm, L, 2, 2, block, halo, prec, band)
    plan = _plan(grid, dmm, L, 2, 2, block, halo, prec, band, P.MPA_SHIFT_AUTO)
    assert plan.info()["shift"] == sh
    plan.close()
    for z0 in (0.5 - 2 * L, 1.0 - 2 * L):
        say("shifted", block, prec, z0, sh)
        got = _run_mpa(a, grid, dmm, L, 2, 2, block, halo, prec, z0, z0 + 4 * L, band, sh)
        ref = O.mpa_propagate(a, grid.dt, dmm, L, 2, 2, z0, z0 + 4 * L, block, halo, sh)
        assert rel_l2(got, ref) < TOL[prec]


@pytest.mark.parametrize("nit", [1, 3, 4, 5])
@pytest.mark.parametrize("M", [1, 3])
def test_sweeps_and_nodes(nit, M):
    grid, a, band, halo, L = _blocked_case(2048, n=1 << 13, bits=8)
    dmm = dm_map(beta3=0.1)
    for prec in (1, 0):
        say("sweeps", nit, "M", M, prec)
        got = _run_mpa(a, grid, dmm, L, M, nit, 2048, halo, prec, 0.0, 2 * L, band)
        ref = O.mpa_propagate(a, grid.dt, dmm, L, M, nit, 0.0, 2 * L, 2048, halo)
        assert rel_l2(got, ref) < TOL[prec]


def test_linear_exactness_on_gpu():
    """sigma = 0: the GPU long step is exact linear propagation."""
    w = WORKLOADS["dm1ch_n4096_f64"]
    a = w.field()
    dmm = dm_map(beta3=0.3, sigma=0.0, gamma=0.05, z_amp=0.0)
    say("linear exactness")
    got = _run_mpa(a, w.grid, dmm, 0.25, 5, 2, 0, 0, 1, 0.0, 0.25)
    ref = O.linear_step(a, O.omega_grid(w.grid.n, w.grid.dt), 20.0, 0.3, 0.05, 0.25)
    assert rel_l2(got, ref) < 1e-12


def test_resume_step_and_determinism():
    import paper_1101_0086_amd as P
    grid, a, band, halo, L = _blocked_case(1024, n=1 << 14, bits=16)
    dmm = dm_map(beta3=0.1)
    say("determinism")
    plan = P.MPAPlan(grid.n, grid.dt, dmm, L, 2, 2, 1024, halo, 0, band)
    x1 = to_dev(a, 0)
    plan.propagate(x1, 0.0, 6 * L)
    x2 = to_dev(a, 0)
    plan.propagate(x2, 0.0, 3 * L)
    plan.propagate(x2, 3 * L, 6 * L)
    x3 = to_dev(a, 0)
    for m in range(6):
        plan.step(x3, m * L)
    r1, r2, r3 = to_host(x1), to_host(x2), to_host(x3)
    plan.close()
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)


@pytest.mark.parametrize("name,over,prec", [
    ("wdm8_n262144_f32", None, 0),
    ("wdm32_n4194304_f32", None, 0),
    ("wdm32_n4194304_f32", None, 1),
    # the autotuner's picks at the same dz: 50 % and 75 % overlaps
    ("wdm8_n262144_f32", dict(block=2048, halo=512, L=3.125e-4, M=5), 0),
    ("wdm8_n262144_f32", dict(block=4096, halo=1536, L=6.25e-4, M=10), 0),
    ("wdm32_n4194304_f32", dict(block=4096, halo=1024, L=1.5625e-5, M=2, shift=0), 0),
    ("wdm32_n4194304_f32", dict(block=4096, halo=512, L=7.8125e-6, M=1, shift=0), 0),
    # shifted windows at the same dz
    ("wdm32_n4194304_f32", dict(block=4096, halo=512, L=1.5625e-5, M=2, shift=96), 0),
    ("wdm32_n4194304_f32", dict(block=2048, halo=256, L=7.8125e-6, M=1, shift=48), 0),
    # blocks above 4096 (four-step transforms, node order), the autotuner's shapes at the same dz
    ("wdm32_n4194304_f32", dict(block=8192, halo=2048, L=6.25e-5, M=8, shift=384), 0),
    ("wdm32_n4194304_f32", dict(block=16384, halo=4096, L=1.25e-4, M=16, shift=769), 0),
    ("wdm32_n4194304_f32", dict(block=32768, halo=8192, L=2.5e-4, M=32, shift=1538), 0),
    ("wdm32_n4194304_f32", dict(block=16384, halo=2048, L=6.25e-5, M=8, shift=384), 1),
])
def test_full_size_sampled_blocks(name, over, prec):
    """The benchmark's 2^18-mode 8-channel workload and the 2^22-mode
    32-channel QPSK workload (the largest configuration) in their launch
    configurations (4096-blocks, 512-halo) and in the wider-overlap
    configurations and blocks of 8192..32768 the autotuner tries at the same
    dz: one long step on the GPU, three blocks (first, middle, ragged last)
    recomputed by the oracle one at a time, roll-off included."""
    import dataclasses
    w = WORKLOADS[name]
    if over:
        w = dataclasses.replace(w, mpa=dataclasses.replace(w.mpa, **over))
    s = w.mpa
    a = w.field()
    say("full size sampled blocks", name, w.grid.n, over, prec)
    got = _run_mpa(a, w.grid, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, prec, 0.0, s.L,
                   s.omega_band, s.shift)
    parts = O.block_partition(w.grid.n, s.block, s.halo, s.shift)
    omega_b = O.omega_grid(s.block, w.grid.dt)
    taper = O.block_taper(s.block, s.halo)
    b2, b3 = w.dmmap.beta2[0], w.dmmap.beta3[0]
    mask = O.block_mask(omega_b, b2, b3, s.L, s.halo, w.grid.dt, s.shift)
    lead = s.halo + s.shift
    for b in (0, len(parts) // 2, len(parts) - 1):
        w0, c0, clen = parts[b]
        idx = (w0 + np.arange(s.block)) % w.grid.n
        res = O.mpa_long_step(a[idx] * taper, omega_b, b2, b3, w.dmmap.sigma[0], w.dmmap.gamma,
                              s.L, s.M, s.n_iter, out_mask=mask)
        ref = res[lead:lead + clen]
        assert rel_l2(got[c0:c0 + clen], ref) < TOL[prec], b


def test_maximum_size_sampled_blocks():
    """The largest field a plan accepts, 2^30 modes in FP32 (8 GiB, 349526
    blocks of 4096 with a ragged 1024-sample last core), in the benchmark's
    launch configuration: the 2^18-mode 8-channel field repeated 4096 times
    (a WDM pulse train of the same structure), one long step, three blocks
    (first, middle, last) recomputed by the oracle one at a time."""
    import torch

    import paper_1101_0086_amd as P
    w = WORKLOADS["wdm8_n262144_f32"]
    s = w.mpa
    n = 1 << 30
    a = w.field()
    say("maximum size sampled blocks", n)
    plan = P.MPAPlan(n, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, 0, s.omega_band)
    assert plan.info()["n_blocks"] == -(-n // (s.block - 2 * s.halo))
    x = torch.from_numpy(a.astype(np.complex64)).to("cuda:0").repeat(n // a.size)
    plan.propagate(x, 0.0, s.L)
    parts = O.block_partition(n, s.block, s.halo)
    omega_b = O.omega_grid(s.block, w.grid.dt)
    taper = O.block_taper(s.block, s.halo)
    b2, b3 = w.dmmap.beta2[0], w.dmmap.beta3[0]
    mask = O.block_mask(omega_b, b2, b3, s.L, s.halo, w.grid.dt)
    checks = []
    for b in (0, len(parts) // 2, len(parts) - 1):
        w0, c0, clen = parts[b]
        idx = (w0 + np.arange(s.block)) % n
        res = O.mpa_long_step(a[idx % a.size] * taper, omega_b, b2, b3, w.dmmap.sigma[0], w.dmmap.gamma,
                              s.L, s.M, s.n_iter, out_mask=mask)
        got = x[c0:c0 + clen].cpu().numpy().astype(np.complex128)
        checks.append((b, clen, rel_l2(got, res[s.halo:s.halo + clen])))
    plan.close()
    del x
    assert checks[-1][1] == 1024
    for b, _, e in checks:
        assert e < TOL_F32, (b, e)
