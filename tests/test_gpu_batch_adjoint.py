"""Batched reverse pass (mpa_batch_propagate_checkpointed / mpa_batch_adjoint
through the C ABI).

* every instance's field gradient equals that of mpa_adjoint on a plan of its
  own with the instance's sigma (bitwise: the reverse kernel runs the same
  per-block arithmetic, only the work list and the grid differ), in both
  precisions, over a range that crosses an amplifier and a map-period
  boundary (two checkpoints), with and without inner checkpoints, and with
  distributed gain;
* the shared parameter derivatives are the sum of the per-instance ones,
  the sigma derivative weighted by each instance's sigma scale (the sums are
  taken in another order, so to 1e-12 of their norm);
* an FP64 batch matches the FP64 oracle's gradients instance by instance;
* the torch.autograd binding over a batch plan returns exactly the C ABI's
  gradients.

Loss l = sum over instances of sum |A_i(z1) - target_i|^2, so
G(A_i(z1)) = 2 (A_i(z1) - target_i).
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import rel_l2, say, to_dev, to_host
from workloads import Grid, dm_map
from workloads.wdm import _fast_wdm_field

pytestmark = pytest.mark.gpu

DT = 10.0 / 1024
BAND = 145.0


def _case(ns, seed, block):
    halo = block // 8
    rate = O.halo_rate(BAND, 20.0, 0.1)
    k = math.ceil(0.5 / (0.25 * halo * DT / rate))
    L = 0.5 / k
    rng = np.random.default_rng(seed)
    fields = [_fast_wdm_field(Grid(n, DT), n // 1024, 8, "ook", np.random.default_rng(seed + i))
              for i, n in enumerate(ns)]
    g_out = [0.1 * (rng.normal(size=n) + 1j * rng.normal(size=n)) for n in ns]
    return fields, g_out, halo, L


@pytest.mark.parametrize("prec,store_steps,gain", [(0, 0, False), (0, 2, False), (1, 0, False), (1, 2, False),
                                                   (0, 0, True)])
def test_batch_adjoint_equals_single_plans(prec, store_steps, gain):
    import paper_1101_0086_amd as P
    from workloads.wdm import DMMap
    ns = [8192, 4096, 16384, 2048]
    scales = [1.0, 0.5, 2.0, 0.8]
    block = 2048
    fields, g_out, halo, L = _case(ns, 5, block)
    dmm = dm_map(beta3=0.1)
    if gain:                                  # distributed gain across the amplifier at 1.0
        dmm = DMMap(**{**dmm.__dict__, "raman_g0": 0.2, "raman_alpha": 3.0})
    z0, z1 = 1.0 - 3 * L, 1.0 + 2 * L       # amplifier and period start at 1.0
    say("batch adjoint vs single plans", prec, store_steps, ns)
    bp = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, block, halo, prec, BAND, sigma_scale=scales)
    assert bp.checkpoint_count(z0, z1) == 2
    x = to_dev(np.concatenate(fields), prec)
    ck = bp.propagate_checkpointed(x, z0, z1)
    g = to_dev(np.concatenate(g_out), prec)
    pg = bp.adjoint(ck, g, z0, z1, store_steps).cpu().numpy()
    got_x = [to_host(v) for v in bp.split(x)]
    got_g = [to_host(v) for v in bp.split(g)]
    bp.close()
    ref_p = np.zeros((3, 2))
    for a, go, n, sc, gx, gg in zip(fields, g_out, ns, scales, got_x, got_g):
        p = P.MPAPlan(n, DT, dmm.with_sigma(sc), L, 2, 2, block, halo, prec, BAND)
        y = to_dev(a, prec)
        c1 = p.propagate_checkpointed(y, z0, z1)
        h = to_dev(go, prec)
        q = p.adjoint(c1, h, z0, z1, store_steps).cpu().numpy()
        p.close()
        assert np.array_equal(to_host(y), gx)
        assert np.array_equal(to_host(h), gg), n
        ref_p[0] += sc * q[0]
        ref_p[1:] += q[1:]
    err = np.linalg.norm(pg - ref_p) / np.linalg.norm(ref_p)
    assert err < 1e-12, (err, pg, ref_p)


@pytest.mark.parametrize("prec", [0, 1])
def test_large_batch_adjoint_equals_single_plans(prec):
    """A batch of 40 fields of 11 blocks (440 work items, more than the CUs:
    the reverse launch deals several items to each workgroup, which reuses
    its LDS twiddle table and node store) gives bitwise the field gradients
    of per-field plans (11 items each, one per workgroup)."""
    import paper_1101_0086_amd as P
    ns = [16384] * 40
    scales = [1.0] * 40
    block = 2048
    fields, g_out, halo, L = _case(ns, 23, block)
    dmm = dm_map(beta3=0.1)
    z0, z1 = 0.0, 2 * L
    say("large batch adjoint", prec)
    bp = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, block, halo, prec, BAND, sigma_scale=scales)
    assert bp.info()["work_items"] == 440
    x = to_dev(np.concatenate(fields), prec)
    ck = bp.propagate_checkpointed(x, z0, z1)
    g = to_dev(np.concatenate(g_out), prec)
    pg = bp.adjoint(ck, g, z0, z1).cpu().numpy()
    got_g = [to_host(v) for v in bp.split(g)]
    bp.close()
    ref_p = np.zeros((3, 2))
    for i in (0, 17, 39):
        p = P.MPAPlan(ns[i], DT, dmm, L, 2, 2, block, halo, prec, BAND)
        y = to_dev(fields[i], prec)
        c1 = p.propagate_checkpointed(y, z0, z1)
        h = to_dev(g_out[i], prec)
        p.adjoint(c1, h, z0, z1)
        p.close()
        assert np.array_equal(to_host(h), got_g[i]), i
    assert np.all(np.isfinite(pg))


def test_batch_adjoint_fp64_matches_oracle():
    import paper_1101_0086_amd as P
    ns = [4096, 2048, 8192]
    scales = [1.0, 1.6, 0.7]
    block = 1024
    fields, g_out, halo, L = _case(ns, 17, block)
    dmm = dm_map(beta3=0.1)
    z0, z1 = 0.5 - 2 * L, 0.5 + L           # span change at 0.5
    say("batch adjoint fp64 vs oracle", ns)
    bp = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, block, halo, P.MPA_C128, BAND, sigma_scale=scales)
    x = to_dev(np.concatenate(fields), 1)
    ck = bp.propagate_checkpointed(x, z0, z1)
    g = to_dev(np.concatenate(g_out), 1)
    pg = bp.adjoint(ck, g, z0, z1).cpu().numpy()
    got_g = [to_host(v) for v in bp.split(g)]
    bp.close()
    ref_p = np.zeros((3, 2))
    for a, go, sc, gg in zip(fields, g_out, scales, got_g):
        ga, gs, g2, g3 = O.mpa_propagate_vjp(a, DT, dmm.with_sigma(sc), L, 2, 2, z0, z1, go, block, halo)
        assert rel_l2(gg, ga) < 1e-10
        ref_p += np.stack([sc * gs, g2, g3])
    err = np.linalg.norm(pg - ref_p) / np.linalg.norm(ref_p)
    assert err < 1e-9, (err, pg, ref_p)


def test_batch_adjoint_empty_range():
    import paper_1101_0086_amd as P
    ns = [2048, 4096]
    fields, g_out, halo, L = _case(ns, 3, 1024)
    bp = P.MPABatchPlan(ns, DT, dm_map(), L, 2, 2, 1024, halo, P.MPA_C64, BAND)
    assert bp.checkpoint_count(0.25, 0.25) == 0
    g = to_dev(np.concatenate(g_out), 0)
    before = to_host(g)
    import torch
    pg = bp.adjoint(torch.empty((0, bp.n), dtype=g.dtype, device=g.device), g, 0.25, 0.25)
    bp.close()
    assert np.array_equal(to_host(g), before)
    assert not pg.cpu().numpy().any()


def test_batch_autograd_binding():
    """The torch.autograd binding over a batch plan returns exactly the
    gradients of mpa_batch_adjoint through the C ABI."""
    import torch

    import paper_1101_0086_amd as P
    from paper_1101_0086_amd.autograd import propagate
    ns = [4096, 2048, 8192]
    scales = [1.0, 1.4, 0.6]
    fields, _, halo, L = _case(ns, 23, 1024)
    dmm = dm_map(beta3=0.1)
    z0, z1 = 1.0 - 2 * L, 1.0 + 3 * L
    say("batch autograd")
    bp = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, 1024, halo, P.MPA_C64, BAND, sigma_scale=scales)
    a = np.concatenate(fields)
    x = to_dev(a, 0).requires_grad_(True)
    sig = torch.tensor(dmm.sigma, dtype=torch.float64, requires_grad=True)
    b3 = torch.tensor(dmm.beta3, dtype=torch.float64, requires_grad=True)
    out = propagate(bp, x, z0, z1, sigma=sig, beta3=b3)
    loss = (out.real ** 2 + out.imag ** 2).sum()
    loss.backward()
    y = to_dev(a, 0)
    ck = bp.propagate_checkpointed(y, z0, z1)
    assert torch.equal(y, out.detach())
    g = 2 * y
    pg = bp.adjoint(ck, g, z0, z1)
    bp.close()
    assert torch.equal(x.grad, g)
    assert torch.equal(sig.grad, pg[0].cpu()) and torch.equal(b3.grad, pg[2].cpu())


def test_batch_kept_inputs_equal_the_recomputing_pass():
    """mpa_batch_adjoint_keep_inputs: field gradients and parameter
    derivatives bitwise those of the recomputing reverse pass."""
    import paper_1101_0086_amd as P
    ns = [4096, 8192, 2048]
    fields, g_out, halo, L = _case(ns, 23, 1024)
    dmm = dm_map(beta3=0.1)
    z0, z1 = 0.5 - 2 * L, 0.5 + 3 * L
    out = []
    for keep in (0, 1 << 30):
        say("batch kept inputs", keep)
        bp = P.MPABatchPlan(ns, DT, dmm, L, 2, 2, 1024, halo, P.MPA_C64, BAND, sigma_scale=[1.0, 1.3, 0.8])
        bp.keep_inputs(keep)
        x = to_dev(np.concatenate(fields), 0)
        ck = bp.propagate_checkpointed(x, z0, z1)
        g = to_dev(np.concatenate(g_out), 0)
        pg = bp.adjoint(ck, g, z0, z1).cpu().numpy()
        out.append((to_host(x), to_host(g), pg))
        bp.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
