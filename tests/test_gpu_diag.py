"""Failure detection through the C ABI: the non-finite scan of a field
(MPA_ENONFINITE) and the Picard residuals of a long step (MPA_EDIVERGE when
the sweeps stop contracting), against the oracle's iterates of the same
long step."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_util import say, to_dev
from workloads import WORKLOADS, dm_map

pytestmark = pytest.mark.gpu


def _oracle_residuals(a, dt, dmmap, L, M, nit, m):
    """||A^(k) - A^(k-1)|| / ||A^(k)||, k = 1..nit, A^(k) the oracle's long step m
    with k sweeps (A^(0): no sweep, the linear step)."""
    outs = [O.mpa_step(a, dt, dmmap, L, M, k, m) for k in range(nit + 1)]
    return [float(np.linalg.norm(outs[k] - outs[k - 1]) / np.linalg.norm(outs[k])) for k in range(1, nit + 1)]


@pytest.mark.parametrize("prec", [1, 0])
def test_check_field(prec):
    import paper_1101_0086_amd as P
    from paper_1101_0086_amd import _lib
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    plan = P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, 0, 0, prec)
    a = w.field()
    say("check field", prec)
    plan.check_field(to_dev(a, prec))
    for bad in (np.nan, np.inf, -np.inf):
        b = a.copy()
        b[1234] = complex(0.1, bad)
        with pytest.raises(P.MPAError) as e:
            plan.check_field(to_dev(b, prec))
        assert e.value.status == _lib.MPA_ENONFINITE
    plan.close()


def test_picard_residuals_match_the_oracle_and_contract():
    """The 4096-mode full-window FP64 plan with 4 sweeps: the residuals of the
    long step at z = 0.4 equal the oracle's and fall geometrically."""
    import paper_1101_0086_amd as P
    from paper_1101_0086_amd import _lib
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    nit = 4
    a = w.field()
    m = int(round(0.4 / s.L))
    ref = _oracle_residuals(a, w.grid.dt, w.dmmap, s.L, s.M, nit, m)
    plan = P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, s.L, s.M, nit, 0, 0, P.MPA_C128)
    x = to_dev(a, 1)
    say("picard residuals")
    st, got = plan.picard_residuals(x, m * s.L, nit)
    plan.close()
    assert st == _lib.MPA_OK
    assert np.array_equal(x.cpu().numpy(), a)                 # the field is left unchanged
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-8 * r, (got, ref)
    assert all(ref[k] < 0.1 * ref[k - 1] for k in range(1, nit))


def test_picard_residuals_blocked_fp32():
    """The 2^18-mode bench field in its launch configuration (4096-blocks,
    FP32 node work): the two residuals fall."""
    import paper_1101_0086_amd as P
    from paper_1101_0086_amd import _lib
    w = WORKLOADS["wdm8_n262144_f32"]
    s = w.mpa
    plan = P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, s.L, s.M, 3, s.block, s.halo, P.MPA_C64, s.omega_band)
    say("picard residuals blocked")
    st, got = plan.picard_residuals(to_dev(w.field(), 0), 0.0, 3)
    plan.close()
    assert st == _lib.MPA_OK and got[1] < got[0] and got[2] < got[1], got


def test_picard_divergence_is_detected():
    """A 500 times stronger nonlinearity (nonlinear phase of several radians
    per long step): the oracle's residuals grow, and the plan reports
    MPA_EDIVERGE with the same residuals."""
    import paper_1101_0086_amd as P
    from paper_1101_0086_amd import _lib
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    nit = 4
    dmm = dm_map(beta3=0.0, sigma=500.0)
    a = w.field()
    ref = _oracle_residuals(a, w.grid.dt, dmm, s.L, s.M, nit, 0)
    assert any(ref[k] >= ref[k - 1] for k in range(1, nit)), ref
    plan = P.MPAPlan(w.grid.n, w.grid.dt, dmm, s.L, s.M, nit, 0, 0, P.MPA_C128)
    say("picard divergence")
    st, got = plan.picard_residuals(to_dev(a, 1), 0.0, nit)
    plan.close()
    assert st == _lib.MPA_EDIVERGE, (st, got, ref)
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-6 * r, (got, ref)
