"""Oracle gradients pinned by central finite differences of the forward
oracle (loss = sum |A_out - A_target|^2, complex directions for the field,
scalar steps for sigma, beta2, beta3)."""
import numpy as np
import pytest

import oracle as O
from oracle import adjoint as AD
from workloads import Grid, dm_map, wdm_field


def _loss(out, target):
    return float(np.sum(np.abs(out - target) ** 2))


def _check(fwd, vjp_val, x0, direction, eps, rtol):
    lp, lm = fwd(x0 + eps * direction), fwd(x0 - eps * direction)
    fd = (lp - lm) / (2 * eps)
    assert abs(fd - vjp_val) <= rtol * max(abs(fd), 1e-12), (fd, vjp_val)


def test_long_step_vjp_matches_finite_differences():
    rng = np.random.default_rng(0)
    n, dt = 64, 0.3
    omega = O.omega_grid(n, dt)
    a0 = 0.5 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    target = rng.normal(size=n) + 1j * rng.normal(size=n)
    mask = np.linspace(1.0, 0.3, n)
    args = dict(beta2=0.7, beta3=0.2, sigma=1.3, gamma=0.05, L=0.4, M=3, n_iter=3)

    def run(a=a0, **kw):
        p = dict(args, **kw)
        return O.mpa_long_step(a, omega, p["beta2"], p["beta3"], p["sigma"], p["gamma"], p["L"],
                               p["M"], p["n_iter"], out_mask=mask)

    out = run()
    g_out = 2 * (out - target)
    g_a, d_s, d_b2, d_b3 = AD.mpa_long_step_vjp(a0, omega, args["beta2"], args["beta3"], args["sigma"],
                                                args["gamma"], args["L"], args["M"], args["n_iter"],
                                                g_out, out_mask=mask)
    for _ in range(3):
        d = rng.normal(size=n) + 1j * rng.normal(size=n)
        _check(lambda a: _loss(run(a=a), target), float(np.real(np.vdot(g_a, d))), a0, d, 1e-6, 1e-6)
    for name, val in (("sigma", d_s), ("beta2", d_b2), ("beta3", d_b3)):
        _check(lambda v, name=name: _loss(run(**{name: v}), target), val, args[name], 1.0, 1e-6, 1e-6)


@pytest.mark.parametrize("shift", [0, 7])
def test_blocked_and_marched_vjp_matches_finite_differences(shift):
    """Across the span change; with and without a window shift (the shifted
    roll-off's beta derivative and the shifted core positions)."""
    rng = np.random.default_rng(1)
    n, dt, B, H = 1024, 10 / 512, 256, 32
    a0 = wdm_field(Grid(n, dt), 4, 2, "ook", rng)
    target = a0 * 0.9 + 0.01 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    L = 0.5 / 8000
    dmm = dm_map(beta3=0.1)
    z0, z1 = 0.5 - 2 * L, 0.5 + 2 * L            # across the span change

    def run(a=a0, dmm=dmm):
        return O.mpa_propagate(a, dt, dmm, L, 2, 2, z0, z1, B, H, shift)

    out = run()
    g_a, g_sigma, g_beta2, g_beta3 = AD.mpa_propagate_vjp(a0, dt, dmm, L, 2, 2, z0, z1, 2 * (out - target), B, H,
                                                          shift)
    d = rng.normal(size=n) + 1j * rng.normal(size=n)
    _check(lambda a: _loss(run(a=a), target), float(np.real(np.vdot(g_a, d))), a0, d, 1e-6, 1e-6)
    for span in (0, 1):
        for field, grad in (("sigma", g_sigma), ("beta2", g_beta2), ("beta3", g_beta3)):
            def f(v, span=span, field=field):
                vals = list(getattr(dmm, field))
                vals[span] = v
                return _loss(run(dmm=dmm.__class__(**{**dmm.__dict__, field: tuple(vals)})), target)
            _check(f, grad[span], getattr(dmm, field)[span], 1.0, 1e-5, 1e-5)


def test_gain_enters_the_gradient():
    rng = np.random.default_rng(2)
    n, dt = 512, 10 / 256
    a0 = wdm_field(Grid(n, dt), 2, 1, "ook", rng)
    dmm = dm_map(beta3=0.0, z_amp=0.5)
    L = 0.25
    out = O.mpa_propagate(a0, dt, dmm, L, 2, 2, 0.25, 0.75)
    g_a, _, _, _ = AD.mpa_propagate_vjp(a0, dt, dmm, L, 2, 2, 0.25, 0.75, 2 * out)
    d = rng.normal(size=n) + 1j * rng.normal(size=n)
    _check(lambda a: _loss(O.mpa_propagate(a, dt, dmm, L, 2, 2, 0.25, 0.75), 0 * a0),
           float(np.real(np.vdot(g_a, d))), a0, d, 1e-6, 1e-6)


def _span_fd(run, dmm, grads, target, rtol, spans):
    for span in spans:
        for field, grad in zip(("sigma", "beta2", "beta3"), grads):
            def f(v, span=span, field=field):
                vals = list(getattr(dmm, field))
                vals[span] = v
                return _loss(run(dmm=dmm.__class__(**{**dmm.__dict__, field: tuple(vals)})), target)
            _check(f, grad[span], getattr(dmm, field)[span], 1.0, 1e-5, rtol)


def test_step_weights_are_the_derivatives_of_the_step_coefficients():
    """sum_s beta2_s len[s] and sum_s sigma_s w[s] rebuild the node integrals
    and node sigmas of every boundary-crossing step (two and three spans in
    one step, a node on a boundary and boundaries between nodes); steps
    inside one span get len = j dz, w = 1."""
    from oracle.nlse import long_step_spans, step_coefficients
    dmm = dm_map(beta3=0.1, beta2=(20.0, -7.0, -19.8), seg=(0.5, 0.05, 0.45))
    dmm = dmm.__class__(**{**dmm.__dict__, "sigma": (1.0, 3.0, 2.0)})
    three = 0
    for L, M in ((1.0 / 7.0, 6), (1.0 / 7.0, 3), (0.125, 4), (0.1, 2)):
        crossing = 0
        for m in range(int(round(1.0 / L))):
            lens, ws = AD.step_weights(dmm, L, M, m)
            spans = long_step_spans(dmm, L, m)
            if len(spans) == 1:
                assert np.allclose(lens[spans[0]], (L / M) * np.arange(M + 1), rtol=0, atol=1e-15)
                assert np.all(ws[spans[0]] == 1.0) and np.sum(ws) == M + 1
                continue
            crossing += 1
            three += len(spans) == 3
            (b2, b3), sig = step_coefficients(dmm, L, M, m)
            assert np.allclose(np.asarray(dmm.beta2) @ lens, b2, rtol=0, atol=1e-13)
            assert np.allclose(np.asarray(dmm.beta3) @ lens, b3, rtol=0, atol=1e-13)
            assert np.allclose(np.asarray(dmm.sigma) @ ws, sig, rtol=0, atol=1e-15)
            assert np.allclose(ws.sum(axis=0), 1.0) and np.allclose(lens.sum(axis=0), (L / M) * np.arange(M + 1))
        assert crossing >= 1
    assert three >= 1


def test_vjp_across_a_boundary_on_a_node_matches_finite_differences():
    """Full window, L = 1/7, M = 6: the step [3/7, 4/7] crosses z = 0.5 with
    node 3 on it (sigma there the mean of both spans)."""
    rng = np.random.default_rng(3)
    n, dt = 256, 10 / 128
    a0 = wdm_field(Grid(n, dt), 2, 1, "ook", rng)
    target = a0 * 0.9 + 0.01 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    base = dm_map(beta3=0.1)
    dmm = base.__class__(**{**base.__dict__, "sigma": (1.0, 2.0)})
    L, z0, z1 = 1.0 / 7.0, 2.0 / 7.0, 5.0 / 7.0

    def run(a=a0, dmm=dmm):
        return O.mpa_propagate(a, dt, dmm, L, 6, 2, z0, z1)

    out = run()
    g_a, g_sigma, g_beta2, g_beta3 = AD.mpa_propagate_vjp(a0, dt, dmm, L, 6, 2, z0, z1, 2 * (out - target))
    d = rng.normal(size=n) + 1j * rng.normal(size=n)
    _check(lambda a: _loss(run(a=a), target), float(np.real(np.vdot(g_a, d))), a0, d, 1e-6, 1e-6)
    _span_fd(run, dmm, (g_sigma, g_beta2, g_beta3), target, 1e-5, (0, 1))


@pytest.mark.parametrize("shift", [0, 5])
def test_blocked_vjp_across_boundaries_matches_finite_differences(shift):
    """Blocked (B = 256, H = 32), L = 1/k with k odd so that the boundary at
    0.5 falls between two nodes of a step; with and without a window shift
    (the roll-off follows the step's mean coefficients)."""
    rng = np.random.default_rng(4)
    n, dt, B, H = 1024, 10 / 512, 256, 32
    a0 = wdm_field(Grid(n, dt), 4, 2, "ook", rng)
    target = a0 * 0.9 + 0.01 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    base = dm_map(beta3=0.1)
    dmm = base.__class__(**{**base.__dict__, "sigma": (1.0, 2.0)})
    k = 8001
    L = 1.0 / k
    m0 = k // 2 - 1
    z0, z1 = m0 * L, (m0 + 3) * L

    def run(a=a0, dmm=dmm):
        return O.mpa_propagate(a, dt, dmm, L, 3, 2, z0, z1, B, H, shift)

    out = run()
    g_a, g_sigma, g_beta2, g_beta3 = AD.mpa_propagate_vjp(a0, dt, dmm, L, 3, 2, z0, z1, 2 * (out - target),
                                                          B, H, shift)
    d = rng.normal(size=n) + 1j * rng.normal(size=n)
    _check(lambda a: _loss(run(a=a), target), float(np.real(np.vdot(g_a, d))), a0, d, 1e-6, 1e-6)
    _span_fd(run, dmm, (g_sigma, g_beta2, g_beta3), target, 1e-5, (0, 1))


def test_vjp_of_a_step_over_three_spans_matches_finite_differences():
    """A map whose middle span (0.05) is shorter than the long step (1/7):
    the step [3/7, 4/7] overlaps three spans."""
    rng = np.random.default_rng(5)
    n, dt = 256, 10 / 128
    a0 = wdm_field(Grid(n, dt), 2, 1, "ook", rng)
    target = a0 * 0.9 + 0.01 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    dmm = dm_map(beta3=0.1, beta2=(20.0, -7.0, -19.8), seg=(0.5, 0.05, 0.45))
    dmm = dmm.__class__(**{**dmm.__dict__, "sigma": (1.0, 3.0, 2.0)})
    L, z0, z1 = 1.0 / 7.0, 3.0 / 7.0, 5.0 / 7.0

    def run(a=a0, dmm=dmm):
        return O.mpa_propagate(a, dt, dmm, L, 3, 2, z0, z1)

    from oracle.nlse import long_step_spans
    assert len(long_step_spans(dmm, L, 3)) == 3
    out = run()
    g_a, g_sigma, g_beta2, g_beta3 = AD.mpa_propagate_vjp(a0, dt, dmm, L, 3, 2, z0, z1, 2 * (out - target))
    d = rng.normal(size=n) + 1j * rng.normal(size=n)
    _check(lambda a: _loss(run(a=a), target), float(np.real(np.vdot(g_a, d))), a0, d, 1e-6, 1e-6)
    _span_fd(run, dmm, (g_sigma, g_beta2, g_beta3), target, 1e-5, (0, 1, 2))


def test_vjp_across_a_boundary_with_distributed_gain_matches_finite_differences():
    """Distributed gain with a step across the span boundary (L = 1/7) and
    an amplifier inside the range (z = 1)."""
    from workloads.wdm import DMMap
    rng = np.random.default_rng(6)
    n, dt = 256, 10 / 128
    a0 = wdm_field(Grid(n, dt), 2, 1, "ook", rng)
    target = a0 * 0.9 + 0.01 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    base = dm_map(beta3=0.1)
    dmm = DMMap(**{**base.__dict__, "sigma": (1.0, 2.0), "raman_g0": 0.2, "raman_alpha": 3.0})
    L, z0, z1 = 1.0 / 7.0, 3.0 / 7.0, 8.0 / 7.0

    def run(a=a0, dmm=dmm):
        return O.mpa_propagate(a, dt, dmm, L, 3, 2, z0, z1)

    out = run()
    g_a, g_sigma, g_beta2, g_beta3 = AD.mpa_propagate_vjp(a0, dt, dmm, L, 3, 2, z0, z1, 2 * (out - target))
    d = rng.normal(size=n) + 1j * rng.normal(size=n)
    _check(lambda a: _loss(run(a=a), target), float(np.real(np.vdot(g_a, d))), a0, d, 1e-6, 1e-6)
    _span_fd(run, dmm, (g_sigma, g_beta2, g_beta3), target, 1e-5, (0, 1))
