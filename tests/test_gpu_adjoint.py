"""GPU reverse pass (mpa_adjoint through the C ABI) against the FP64 oracle
gradient and against central finite differences of the GPU forward.

Loss l = sum |A(z1) - target|^2, so G(A(z1)) = 2 (A(z1) - target); the same
G(A(z1)) array (from the oracle's forward) is handed to both sides.  Cases:
full window and blocked plans, both precisions, ranges across a span change,
an amplifier and a map-period boundary (two checkpoints), the 2^16-mode
4-channel workload at full size (oracle on two long steps, finite
differences over a whole map period), the inner-checkpoint path, the
autograd binding, and the empty range.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import centred_shift, rel_l2, say, to_dev, to_host
from workloads import WORKLOADS, Grid, dm_map, wdm_field

pytestmark = pytest.mark.gpu

# Tolerances.  FP64 plans: every operation is FP64, so the gradient agrees
# with the oracle to rounding (1e-10 as for the forward).  FP32 plans: the
# node evaluations (transforms and nonlinearity) of both the recomputed
# forward and the reverse pass run in FP32 (unit roundoff 6e-8, FFT error
# about 2e-7 relative), the output-sized gradient and the carry in FP64.  The
# field gradient stays within 1e-5.  The parameter derivatives are compared
# as one vector (sigma, beta2, beta3 of every span) relative to its norm:
# within 1e-4 when the loss only looks at the signal band (a target in the
# band), within 1e-3 when the target carries white noise.  Reason for the
# second bound: the FP32 transform of |A|^2 A leaves rounding noise of about
# 1e-7 of its largest value at every frequency, and the beta2 and beta3
# derivatives weight each frequency's product of that increment with its
# adjoint by omega^2 z / 2 and omega^3 z / 6; a white-noise target gives the
# adjoint O(1) content up to |omega| = pi / dt, where the weights exceed the
# band's by (pi / dt / omega_band)^3 (4096 on the 4096-mode case), so the
# noise enters the beta3 derivative at ~1e-7 * 4096 relative.  The FP32
# forward map itself carries that noise, so this is a property of FP32 node
# evaluations, not of the reverse pass (the FP64 plan matches to 1e-9).
TOL_G = {1: 1e-10, 0: 1e-5}
TOL_P = {1: 1e-9, 0: 1e-4}
TOL_P_BROADBAND_F32 = 1e-3


def _target(a, dt, rng, scale, noise, band=None):
    """scale * a plus complex white noise of rms `noise`, or, with `band`,
    the same noise restricted to |omega| <= band (a loss on the signal band)."""
    nz = noise * (rng.normal(size=a.size) + 1j * rng.normal(size=a.size))
    if band is not None:
        omega = 2 * np.pi * np.fft.fftfreq(a.size, dt)
        spec = np.fft.fft(nz)
        spec[np.abs(omega) > band] = 0
        nz = np.fft.ifft(spec)
    return scale * a + nz


def _plan(grid, dmmap, L, M, nit, block, halo, prec, band=0.0, shift=0):
    import paper_1101_0086_amd as P
    return P.MPAPlan(grid.n, grid.dt, dmmap, L, M, nit, block, halo, prec, band, shift=shift)


def _gpu_grad(plan, a, g_out, z0, z1, prec, store_steps=0):
    x = to_dev(a, prec)
    ck = plan.propagate_checkpointed(x, z0, z1)
    g = to_dev(g_out, prec)
    pg = plan.adjoint(ck, g, z0, z1, store_steps)
    return to_host(x), to_host(g), pg.cpu().numpy()


def _compare(prec, got_g, got_p, ref_g, ref_p, broadband=False):
    eg = rel_l2(got_g, ref_g)
    ref_p = np.asarray(ref_p)
    ep = float(np.linalg.norm(got_p - ref_p) / np.linalg.norm(ref_p))
    say("gradient errors", prec, "field", eg, "parameters", ep, "broadband" if broadband else "in band")
    tol_p = TOL_P_BROADBAND_F32 if (broadband and prec == 0) else TOL_P[prec]
    assert eg < TOL_G[prec], ("field gradient", eg)
    assert ep < tol_p, ("parameter derivatives", ep, got_p, ref_p)


def _oracle(a, dt, dmmap, L, M, nit, z0, z1, target, block=0, halo=0, shift=0):
    out = O.mpa_propagate(a, dt, dmmap, L, M, nit, z0, z1, block, halo, shift)
    g_out = 2 * (out - target)
    g, gs, g2, g3 = O.mpa_propagate_vjp(a, dt, dmmap, L, M, nit, z0, z1, g_out, block, halo, shift)
    return out, g_out, g, np.stack([gs, g2, g3])


@pytest.mark.parametrize("prec,band", [(1, None), (0, None), (0, 10.0)])
def test_full_window_across_span_amplifier_and_period(prec, band):
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    a = w.field()
    rng = np.random.default_rng(11)
    target = _target(a, w.grid.dt, rng, 0.8, 0.05, band)
    z0, z1 = 0.4, 1.1                      # span change at 0.5, amplifier and period start at 1.0
    _, g_out, ref_g, ref_p = _oracle(a, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, z0, z1, target)
    say("adjoint full window", prec)
    plan = _plan(w.grid, w.dmmap, s.L, s.M, s.n_iter, 0, 0, prec)
    assert plan.checkpoint_count(z0, z1) == 2
    _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, prec)
    _compare(prec, got_g, got_p, ref_g, ref_p, broadband=band is None)


def _blocked(block, n=1 << 13, ch=4, seed=7):
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


@pytest.mark.parametrize("block,prec,inband", [(512, 1, False), (512, 0, False), (512, 0, True),
                                               (4096, 1, False), (4096, 0, False), (4096, 0, True)])
def test_blocked_across_span_and_amplifier(block, prec, inband):
    grid, a, band, halo, L = _blocked(block)
    dmmap = dm_map(beta3=0.1)
    rng = np.random.default_rng(12)
    target = _target(a, grid.dt, rng, 0.9, 0.02, band if inband else None)
    M, nit = 2, 2
    for z0, z1 in ((0.5 - 2 * L, 0.5 + 2 * L), (1.0 - 2 * L, 1.0 + L)):
        _, g_out, ref_g, ref_p = _oracle(a, grid.dt, dmmap, L, M, nit, z0, z1, target, block, halo)
        say("adjoint blocked", block, prec, z0, z1)
        plan = _plan(grid, dmmap, L, M, nit, block, halo, prec, band)
        _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, prec)
        _compare(prec, got_g, got_p, ref_g, ref_p, broadband=not inband)
        plan.close()


@pytest.mark.parametrize("block,prec", [(512, 1), (4096, 1), (4096, 0)])
def test_shifted_windows(block, prec):
    """Windows shifted against their cores (the shifted roll-off's beta
    derivatives, shifted gather of the window gradients) across the span
    change and an amplifier."""
    grid, a, band, halo, L = _blocked(block)
    dmmap = dm_map(beta3=0.1)
    sh = centred_shift(band, dmmap, L, grid.dt, halo)
    rng = np.random.default_rng(17)
    target = _target(a, grid.dt, rng, 0.9, 0.02, band)
    for z0, z1 in ((0.5 - 2 * L, 0.5 + 2 * L), (1.0 - 2 * L, 1.0 + L)):
        _, g_out, ref_g, ref_p = _oracle(a, grid.dt, dmmap, L, 2, 2, z0, z1, target, block, halo, sh)
        say("adjoint shifted", block, prec, sh, z0, z1)
        plan = _plan(grid, dmmap, L, 2, 2, block, halo, prec, band, sh)
        _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, prec)
        _compare(prec, got_g, got_p, ref_g, ref_p)
        plan.close()


@pytest.mark.parametrize("block,halo", [(512, 192), (1024, 256)])
def test_wide_overlaps(block, halo):
    """75 % and 50 % overlaps (halo 3B/8 and B/4, the autotuner's gradient
    picks): FP32 plans against the oracle across a span change."""
    grid, a, band, _, _ = _blocked(block)
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(0.5 / (0.25 * halo * grid.dt / rate))
    while (0.5 / k) * rate > 0.25 * halo * grid.dt:
        k += 1
    L = 0.5 / k
    dmmap = dm_map(beta3=0.1)
    target = 0.8 * a
    z0, z1 = 0.5 - 2 * L, 0.5 + 2 * L
    _, g_out, ref_g, ref_p = _oracle(a, grid.dt, dmmap, L, 2, 2, z0, z1, target, block, halo)
    say("adjoint wide overlap", block, halo)
    plan = _plan(grid, dmmap, L, 2, 2, block, halo, 0, band)
    _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, 0)
    plan.close()
    _compare(0, got_g, got_p, ref_g, ref_p)


@pytest.mark.parametrize("nit", [1, 3])
def test_sweeps_and_nodes(nit):
    grid, a, band, halo, L = _blocked(1024)
    dmmap = dm_map(beta3=0.1)
    target = 0.5 * a
    M = 3
    z0, z1 = 0.25, 0.25 + 3 * L
    _, g_out, ref_g, ref_p = _oracle(a, grid.dt, dmmap, L, M, nit, z0, z1, target, 1024, halo)
    say("adjoint sweeps", nit)
    plan = _plan(grid, dmmap, L, M, nit, 1024, halo, 1, band)
    _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, 1)
    _compare(1, got_g, got_p, ref_g, ref_p)


@pytest.mark.parametrize("prec,inband", [(1, False), (0, False), (0, True)])
def test_c5_full_size_two_long_steps_against_oracle(prec, inband):
    """2^16 modes, 4 OOK channels, B = 2048, H = 256, L = 2.5e-4, M = 2, two
    sweeps, beta3 = 0.1: the launch configuration of the gradient workload."""
    w = WORKLOADS["wdm4_n65536_f32"]
    s = w.mpa
    a = w.field()
    rng = np.random.default_rng(13)
    target = _target(a, w.grid.dt, rng, 1.0, 0.01, s.omega_band if inband else None)
    z0, z1 = 0.5 - s.L, 0.5 + s.L
    _, g_out, ref_g, ref_p = _oracle(a, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, z0, z1, target, s.block, s.halo)
    say("adjoint c5 two steps", prec)
    plan = _plan(w.grid, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, prec, s.omega_band)
    _, got_g, got_p = _gpu_grad(plan, a, g_out, z0, z1, prec)
    _compare(prec, got_g, got_p, ref_g, ref_p, broadband=not inband)


# Central differences over one map period: (field step, sigma step, beta2
# step, beta3 step, tolerance, relative noise of the loss) per precision.
# FP64: steps that move the dispersion phase of the signal band
# (|omega| <= 65) by ~1e-4 rad over a span (linear regime), differences to
# 1e-6 (field) and 1e-5 (parameters).  FP32: the loss of the FP32 forward
# carries rounding noise (measured: ~7e-8 of the loss, from the field
# differences with a 1e-3 step, 9e-4 off), so the steps are ~100 times
# larger (a 2e-2 field step moves the loss by ~1e-3 of itself; parameter
# steps move the band's phase by ~1e-2 rad) and each difference is allowed
# 1e-4 plus three times its own noise, 1e-7 loss / (2 h |difference|): the
# sigma derivative (~7 against a loss of ~300) resolves to ~6e-4 at h = 1e-2,
# the field and beta derivatives to ~1e-5.
FD = {1: (1e-5, 1e-4, 1e-7, 4e-9, 1e-6, 1e-5, 0.0), 0: (2e-2, 1e-2, 1e-5, 4e-7, 1e-4, 1e-4, 1e-7)}


@pytest.mark.parametrize("prec", [1, 0])
def test_c5_full_period_finite_differences(prec):
    """Directional derivatives over one whole map period (4000 long steps)
    against central differences of the GPU forward in the same precision:
    the field along a random direction, and sigma, beta2, beta3 of both
    spans."""
    import torch
    w = WORKLOADS["wdm4_n65536_f32"]
    s = w.mpa
    a = w.field()
    rng = np.random.default_rng(14)
    target = a * 0.7
    z0, z1 = 0.0, 1.0
    eps, h_sig, h_b2, h_b3, tol_g, tol_p, noise = FD[prec]

    def loss(dmmap, field):
        plan = _plan(w.grid, dmmap, s.L, s.M, s.n_iter, s.block, s.halo, prec, s.omega_band)
        x = to_dev(field, prec)
        plan.propagate(x, z0, z1)
        plan.close()
        return float(np.sum(np.abs(to_host(x) - target) ** 2))

    say("adjoint c5 period: adjoint", prec)
    plan = _plan(w.grid, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, prec, s.omega_band)
    x = to_dev(a, prec)
    ck = plan.propagate_checkpointed(x, z0, z1)
    g = 2 * (x - torch.from_numpy(target).to(device=x.device, dtype=x.dtype))
    pg = plan.adjoint(ck, g, z0, z1).cpu().numpy()
    g = to_host(g)
    plan.close()

    d = rng.normal(size=a.size) + 1j * rng.normal(size=a.size)
    d *= np.linalg.norm(a) / np.linalg.norm(d)
    say("adjoint c5 period: field differences", prec)
    l0 = loss(w.dmmap, a)
    fd = (loss(w.dmmap, a + eps * d) - loss(w.dmmap, a - eps * d)) / (2 * eps)
    ad = float(np.real(np.vdot(g, d)))
    say("field", fd, ad, abs(fd - ad) / abs(fd))
    bad = [] if abs(fd - ad) <= tol_g * abs(fd) + 3 * noise * l0 / (2 * eps) else [("field", fd, ad)]
    for q, field, h in ((0, "sigma", h_sig), (1, "beta2", h_b2), (2, "beta3", h_b3)):
        for span in (0, 1):
            vals = list(getattr(w.dmmap, field))
            plus, minus = list(vals), list(vals)
            plus[span] += h
            minus[span] -= h
            say("adjoint c5 period: differences in", field, span, prec)
            fd = (loss(w.dmmap.__class__(**{**w.dmmap.__dict__, field: tuple(plus)}), a)
                  - loss(w.dmmap.__class__(**{**w.dmmap.__dict__, field: tuple(minus)}), a)) / (2 * h)
            say(field, span, fd, pg[q, span], abs(fd - pg[q, span]) / abs(fd))
            if abs(fd - pg[q, span]) > tol_p * abs(fd) + 3 * noise * l0 / (2 * h):
                bad.append((field, span, fd, pg[q, span]))
    assert not bad, bad


def test_inner_checkpoints_are_bitwise_identical():
    grid, a, band, halo, L = _blocked(512)
    dmmap = dm_map(beta3=0.1)
    g_out = np.random.default_rng(15).normal(size=a.size) + 0j
    z0, z1 = 0.5 - 5 * L, 0.5 + 6 * L
    plan = _plan(grid, dmmap, L, 2, 2, 512, halo, 0, band)
    say("adjoint inner checkpoints")
    _, g_all, p_all = _gpu_grad(plan, a, g_out, z0, z1, 0, store_steps=0)
    for q in (1, 3, 4):
        _, g_q, p_q = _gpu_grad(plan, a, g_out, z0, z1, 0, store_steps=q)
        assert np.array_equal(g_q, g_all) and np.array_equal(p_q, p_all), q


def test_overlapped_recompute_is_bitwise_identical():
    """Four checkpoint segments (two whole map periods of 4836 long steps):
    the automatic rule recomputes each segment's step inputs on a second
    stream while the previous segment is reversed; the gradients equal, bit
    for bit, those of the one-stream schedule (all inputs of a segment kept,
    store_steps = 4836) and of inner checkpoints every 1000 long steps."""
    grid, a, band, halo, L = _blocked(1024)
    dmmap = dm_map(beta3=0.1)
    g_out = np.random.default_rng(19).normal(size=a.size) + 1j * np.random.default_rng(20).normal(size=a.size)
    z0, z1 = 1.0 - 5 * L, 3.0 + 4 * L
    plan = _plan(grid, dmmap, L, 2, 2, 1024, halo, 0, band)
    assert plan.checkpoint_count(z0, z1) == 4
    say("adjoint overlapped recompute")
    _, g_ov, p_ov = _gpu_grad(plan, a, g_out, z0, z1, 0, store_steps=0)
    for q in (int(round(1.0 / L)), 1000):
        _, g_q, p_q = _gpu_grad(plan, a, g_out, z0, z1, 0, store_steps=q)
        assert np.array_equal(g_q, g_ov) and np.array_equal(p_q, p_ov), q
    plan.close()


def test_checkpointed_forward_matches_propagate():
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    a = w.field()
    plan = _plan(w.grid, w.dmmap, s.L, s.M, s.n_iter, 0, 0, 0)
    say("checkpointed forward")
    x = to_dev(a, 0)
    ck = plan.propagate_checkpointed(x, 0.6, 3.2)
    assert ck.shape[0] == 4                 # 0.6, 1, 2, 3
    y = to_dev(a, 0)
    plan.propagate(y, 0.6, 3.2)
    assert np.array_equal(to_host(x), to_host(y))
    y = to_dev(a, 0)
    for k, z in enumerate((1.0, 2.0, 3.0)):
        plan.propagate(y, 0.6 if k == 0 else z - 1.0, z)
        assert np.array_equal(to_host(ck[k + 1]), to_host(y)), z


def test_empty_range_is_identity():
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    import torch
    plan = _plan(w.grid, w.dmmap, s.L, s.M, s.n_iter, 0, 0, 1)
    g0 = np.random.default_rng(16).normal(size=w.grid.n) + 0j
    g = to_dev(g0, 1)
    ck = torch.empty((0, w.grid.n), dtype=torch.complex128, device="cuda:0")
    pg = plan.adjoint(ck, g, 0.5, 0.5).cpu().numpy()
    assert np.array_equal(to_host(g), g0) and not pg.any()


def test_autograd_binding():
    import torch

    from paper_1101_0086_amd.autograd import propagate
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    a = w.field()
    plan = _plan(w.grid, w.dmmap, s.L, s.M, s.n_iter, 0, 0, 1)
    target = torch.from_numpy(0.8 * a).to("cuda:0")
    say("autograd binding")
    x = to_dev(a, 1).requires_grad_(True)
    sig = torch.tensor(w.dmmap.sigma, dtype=torch.float64, requires_grad=True)
    b2 = torch.tensor(w.dmmap.beta2, dtype=torch.float64, requires_grad=True)
    out = propagate(plan, x, 0.3, 1.2, sigma=sig, beta2=b2)
    diff = out - target
    loss = (diff.real ** 2 + diff.imag ** 2).sum()      # backward gives exactly 2 (out - target)
    loss.backward()
    # the same gradient through the C ABI directly
    y = to_dev(a, 1)
    ck = plan.propagate_checkpointed(y, 0.3, 1.2)
    assert torch.equal(y, out.detach())
    g = 2 * (y - target)
    pg = plan.adjoint(ck, g, 0.3, 1.2)
    assert torch.equal(x.grad, g)
    assert torch.equal(sig.grad, pg[0].cpu()) and torch.equal(b2.grad, pg[1].cpu())
    with pytest.raises(ValueError):
        propagate(plan, x, 0.3, 1.2, sigma=sig * 2)


def test_kept_inputs_equal_the_recomputing_pass():
    """mpa_adjoint_keep_inputs: the checkpointed forward keeps every step
    input (field and checkpoints bitwise those of the plain checkpointed
    forward), and the reverse over the same range and checkpoints, which then
    recomputes nothing, is bitwise the recomputing reverse; a forward of
    another field moves the kept inputs to its own checkpoints, and the
    first run's reverse then recomputes (still bitwise); a budget smaller
    than the range keeps nothing."""
    import torch
    grid, a, band, halo, L = _blocked(1024)
    dmmap = dm_map(beta3=0.1)
    z0, z1 = 0.5 - 2 * L, 1.0 + L                 # two checkpoints (map period at 1.0)
    rng = np.random.default_rng(21)
    g_out = 0.1 * (rng.normal(size=a.size) + 1j * rng.normal(size=a.size))
    say("kept inputs")
    ref = _plan(grid, dmmap, L, 2, 2, 1024, halo, 0, band)
    x = to_dev(a, 0)
    ck_ref = ref.propagate_checkpointed(x, z0, z1)
    g_ref = to_dev(g_out, 0)
    pg_ref = ref.adjoint(ck_ref, g_ref, z0, z1)
    x_ref, ck_ref, g_ref, pg_ref = to_host(x), ck_ref.cpu().numpy(), to_host(g_ref), pg_ref.cpu().numpy()
    ref.close()
    plan = _plan(grid, dmmap, L, 2, 2, 1024, halo, 0, band)
    plan.keep_inputs(1 << 30)
    x1 = to_dev(a, 0)
    ck1 = plan.propagate_checkpointed(x1, z0, z1)
    assert np.array_equal(to_host(x1), x_ref) and np.array_equal(ck1.cpu().numpy(), ck_ref)
    g = to_dev(g_out, 0)
    pg = plan.adjoint(ck1, g, z0, z1).cpu().numpy()
    assert np.array_equal(to_host(g), g_ref) and np.array_equal(pg, pg_ref)
    x2 = to_dev(0.9 * a, 0)
    ck2 = plan.propagate_checkpointed(x2, z0, z1)
    g = to_dev(g_out, 0)
    pg = plan.adjoint(ck1, g, z0, z1).cpu().numpy()
    assert np.array_equal(to_host(g), g_ref) and np.array_equal(pg, pg_ref)
    plan.keep_inputs(1)
    x3 = to_dev(a, 0)
    ck3 = plan.propagate_checkpointed(x3, z0, z1)
    g = to_dev(g_out, 0)
    pg = plan.adjoint(ck3, g, z0, z1).cpu().numpy()
    assert np.array_equal(to_host(g), g_ref) and np.array_equal(pg, pg_ref)
    plan.close()
    del ck2
    torch.cuda.synchronize()
