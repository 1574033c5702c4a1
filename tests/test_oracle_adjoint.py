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
