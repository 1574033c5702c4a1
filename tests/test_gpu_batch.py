"""Batched launches over instances of different lengths, and captured HIP
graphs, through the C ABI.

* every instance of a batch equals the same field run alone (bitwise: the
  batch kernel does the same arithmetic per block, only the work list
  differs), with a per-instance sigma;
* an FP64 batch matches the oracle instance by instance;
* a captured graph replayed several times, with eager work and
  synchronisations between replays, matches the eager result every time;
* the benchmark's 256-instance batch at full size, in its launch
  configuration, on sampled blocks of sampled instances against the oracle.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import centred_shift, TOL_F64, rel_l2, say, to_dev, to_host
from workloads import Grid, dm_map
from workloads.wdm import _fast_wdm_field

pytestmark = pytest.mark.gpu

DT = 10.0 / 1024
BAND = 145.0


def _case(ns, seed=11, block=2048):
    halo = block // 8
    rate = O.halo_rate(BAND, 20.0, 0.1)
    k = math.ceil(0.5 / (0.25 * halo * DT / rate))
    L = 0.5 / k
    fields = [_fast_wdm_field(Grid(n, DT), n // 1024, 8, "ook", np.random.default_rng(seed + i))
              for i, n in enumerate(ns)]
    return fields, block, halo, L


def test_batch_equals_single_runs_bitwise():
    import paper_1101_0086_amd as P
    ns = [8192, 4096, 16384, 8192, 2048]
    scales = [1.0, 0.5, 2.0, 1.3, 0.8]
    fields, block, halo, L = _case(ns)
    dmm = dm_map(beta3=0.1)
    say("batch vs single", ns)
    bp = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, block, halo, P.MPA_C64, BAND, sigma_scale=scales)
    assert bp.info()["work_items"] == sum(-(-n // (block - 2 * halo)) for n in ns)
    x = to_dev(np.concatenate(fields), 0)
    bp.propagate(x, 0.5 - 2 * L, 0.5 + 3 * L)
    got = [to_host(v) for v in bp.split(x)]
    bp.close()
    for a, n, sc, g in zip(fields, ns, scales, got):
        p = P.MPAPlan(n, DT, dmm.with_sigma(sc), L, 2, 2, block, halo, P.MPA_C64, BAND)
        y = to_dev(a, 0)
        p.propagate(y, 0.5 - 2 * L, 0.5 + 3 * L)
        assert np.array_equal(to_host(y), g)
        p.close()


def test_batch_with_shifted_windows_equals_single_runs():
    import paper_1101_0086_amd as P
    ns = [8192, 4096, 16384]
    scales = [1.0, 0.7, 1.6]
    fields, block, halo, L = _case(ns, seed=31)
    dmm = dm_map(beta3=0.1)
    sh = centred_shift(BAND, dmm, L, DT, halo)
    say("batch shifted", ns, sh)
    bp = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, block, halo, P.MPA_C64, BAND, sigma_scale=scales, shift=sh)
    x = to_dev(np.concatenate(fields), 0)
    bp.propagate(x, 0.5 - 2 * L, 0.5 + 3 * L)
    got = [to_host(v) for v in bp.split(x)]
    bp.close()
    for a, n, sc, g in zip(fields, ns, scales, got):
        p = P.MPAPlan(n, DT, dmm.with_sigma(sc), L, 2, 2, block, halo, P.MPA_C64, BAND, shift=sh)
        y = to_dev(a, 0)
        p.propagate(y, 0.5 - 2 * L, 0.5 + 3 * L)
        assert np.array_equal(to_host(y), g)
        p.close()


def test_batch_fp64_matches_oracle():
    import paper_1101_0086_amd as P
    ns = [4096, 8192, 2048]
    scales = [1.0, 1.7, 0.6]
    fields, block, halo, L = _case(ns, seed=21, block=1024)
    dmm = dm_map(beta3=0.1)
    say("batch fp64 vs oracle")
    bp = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, block, halo, P.MPA_C128, BAND, sigma_scale=scales)
    x = to_dev(np.concatenate(fields), 1)
    bp.propagate(x, 1.0 - 2 * L, 1.0 + L)
    got = [to_host(v) for v in bp.split(x)]
    bp.close()
    for a, sc, g in zip(fields, scales, got):
        ref = O.mpa_propagate(a, DT, dmm.with_sigma(sc), L, 2, 2, 1.0 - 2 * L, 1.0 + L, block, halo)
        assert rel_l2(g, ref) < TOL_F64


@pytest.mark.parametrize("batched", [False, True])
def test_graph_replays_match_eager(batched):
    import torch
    import paper_1101_0086_amd as P
    ns = [8192, 4096]
    fields, block, halo, L = _case(ns, seed=31)
    dmm = dm_map(beta3=0.1)
    z0, z1 = 0.5 - 2 * L, 0.5 + L          # odd number of long steps: ends with the copy kernel
    if batched:
        plan = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, block, halo, P.MPA_C64, BAND)
        a0 = np.concatenate(fields)
    else:
        plan = P.MPAPlan(ns[0], DT, dmm, L, 2, 2, block, halo, P.MPA_C64, BAND)
        a0 = fields[0]
    say("graph replay", batched)
    g_buf = to_dev(a0, 0)
    graph = plan.capture(g_buf, z0, z1)
    e_buf = to_dev(a0, 0)
    scratch = torch.zeros(1 << 16, device="cuda:0")
    for rep in range(4):
        graph.launch()
        plan.propagate(e_buf, z0, z1)
        scratch.add_(1.0)                    # eager work of the program between replays
        torch.cuda.synchronize()
        assert np.array_equal(to_host(g_buf), to_host(e_buf)), rep
    graph.close()
    plan.close()


def test_autotuner_picks_a_valid_plan():
    import torch
    import paper_1101_0086_amd as P
    from paper_1101_0086_amd.autotune import autotune
    n = 1 << 15
    a = _fast_wdm_field(Grid(n, DT), 32, 8, "ook", np.random.default_rng(41))
    x = to_dev(a, 0)
    say("autotune")
    dmm = dm_map(beta3=0.1)
    best, cands = autotune(x, DT, dmm, 1.25e-4, 2, BAND, launches=8)
    assert best in cands and all(c.seconds_per_unit_z > 0 for c in cands)
    assert np.array_equal(to_host(x), to_host(to_dev(a, 0)))        # input left unchanged
    plan = P.MPAPlan(n, DT, dmm, best.L, best.M, 2, best.block, best.halo, P.MPA_C64, BAND, shift=best.shift)
    plan.propagate(x, 0.0, 2 * best.L)
    plan.close()


def test_picard_sweeps_chosen_from_the_residual():
    """choose_n_iter: the returned sweep count is the smallest within tol of
    the 5-sweep result; the distances shrink with every sweep until FP64
    rounding; a field 16 times more powerful (nonlinear length 16 times
    shorter) is farther from the fixed point after the same sweeps (the
    floor (L / z_nl)^(n+1)) and never needs fewer sweeps."""
    from paper_1101_0086_amd.autotune import choose_n_iter
    n = 1 << 15
    a = _fast_wdm_field(Grid(n, DT), 32, 8, "ook", np.random.default_rng(42))
    dmm = dm_map(beta3=0.1)
    picks, dists = [], []
    for amp in (1.0, 4.0):
        say("choose_n_iter", amp)
        x = to_dev(amp * a, 1)
        nit, dist = choose_n_iter(x, DT, dmm, 2.5e-4, 2, 4096, 512, BAND, precision=1, tol=1e-12, steps=40)
        assert dist[nit] <= 1e-12 and all(dist[k] > 1e-12 for k in dist if k < nit)
        assert all(dist[k + 1] < dist[k] for k in range(1, 4) if dist[k + 1] > 1e-13)
        picks.append(nit)
        dists.append(dist)
    assert picks[1] >= picks[0]
    assert dists[1][1] > 10 * dists[0][1]


def test_batched_workload_full_size_sampled_blocks():
    """The benchmark's batch at full size (256 instances, N = 2^14..2^18,
    sum N = 2.7e7, 8915 work items) in its launch configuration (4096-blocks,
    512-halo, L = 5e-5, M = 1, two sweeps, FP32, per-instance sigma): one
    batched long step, then the first, middle and last block of four
    instances (the first, the last, the shortest and the longest)
    recomputed by the oracle one at a time, roll-off included."""
    import torch

    import paper_1101_0086_amd as P
    from tests.gpu_util import TOL_F32
    from workloads.wdm import batched_instances
    inst = batched_instances(256, 4)
    ns = [g.n for g, _, _, _ in inst]
    sig = [s for _, _, s, _ in inst]
    dt = inst[0][0].dt
    band = 0.5 * 15 * 40.0 + 5.0
    L, M, nit, B, H = 5e-5, 1, 2, 4096, 512
    dmm = dm_map(beta3=0.1)
    say("batched workload full size", len(ns), sum(ns))
    bp = P.MPABatchPlan(ns, dt, dmm, L, M, nit, B, H, P.MPA_C64, band, sigma_scale=sig)
    assert bp.info()["work_items"] == sum(-(-n // (B - 2 * H)) for n in ns)
    x = torch.from_numpy(np.concatenate([f for _, _, _, f in inst])).to(device="cuda:0", dtype=torch.complex64)
    bp.propagate(x, 0.0, L)
    views = bp.split(x)
    omega_b = O.omega_grid(B, dt)
    taper = O.block_taper(B, H)
    mask = O.block_mask(omega_b, dmm.beta2[0], dmm.beta3[0], L, H, dt)
    picks = sorted({0, len(ns) - 1, int(np.argmin(ns)), int(np.argmax(ns))})
    for i in picks:
        a = inst[i][3]
        n = ns[i]
        got = views[i].cpu().numpy().astype(np.complex128)
        parts = O.block_partition(n, B, H)
        for b in (0, len(parts) // 2, len(parts) - 1):
            w0, c0, clen = parts[b]
            idx = (w0 + np.arange(B)) % n
            res = O.mpa_long_step(a[idx] * taper, omega_b, dmm.beta2[0], dmm.beta3[0], sig[i], dmm.gamma, L, M,
                                  nit, out_mask=mask)
            assert rel_l2(got[c0:c0 + clen], res[H:H + clen]) < TOL_F32, (i, n, b)
    bp.close()
