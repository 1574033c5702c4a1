"""Full-window MPA for windows larger than one workgroup's transform
(four-step transforms, 8192 <= N <= 2^22) through the C ABI: against the
FP64 oracle's full-window MPA (no blocks) at sizes the oracle runs in
seconds, across a span change and an amplifier, both precisions; and the
blocking error of the time-blocked plan measured against it at 2^16 modes."""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import TOL_F32, TOL_F64, rel_l2, say, to_dev, to_host
from workloads import Grid, dm_map, wdm_field

pytestmark = pytest.mark.gpu

TOL = {0: TOL_F32, 1: TOL_F64}


@pytest.mark.parametrize("n,prec", [(1 << 13, 1), (1 << 13, 0), (1 << 14, 1), (1 << 15, 0)])
def test_window_against_oracle(n, prec):
    import paper_1101_0086_amd as P
    dt = 10.0 / 256
    a = wdm_field(Grid(n, dt), n // 256, 1, "ook", np.random.default_rng(51))
    dmm = dm_map(beta3=0.1)
    L, M, nit = 0.05, 4, 2
    z0, z1 = 0.45, 1.1                          # span change at 0.5, amplifier at 1.0
    say("window", n, prec)
    plan = P.MPAPlan(n, dt, dmm, L, M, nit, 0, 0, prec)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    ref = O.mpa_propagate(a, dt, dmm, L, M, nit, z0, z1)
    assert rel_l2(to_host(x), ref) < TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
def test_window_at_2_22_modes(prec):
    """The 1024 x 4096 shape (2^22 modes, rows of 4096 points): one long step
    against the oracle's full-window long step."""
    import paper_1101_0086_amd as P
    from workloads.wdm import _fast_wdm_field
    n, dt = 1 << 22, 10.0 / 4096
    a = _fast_wdm_field(Grid(n, dt), n // 4096, 8, "qpsk", np.random.default_rng(53))
    dmm = dm_map(beta3=0.1)
    L, M, nit = 1e-4, 2, 2
    z0, z1 = 0.2, 0.2 + L
    say("window 2^22", prec)
    plan = P.MPAPlan(n, dt, dmm, L, M, nit, 0, 0, prec)
    x = to_dev(a, prec)
    plan.propagate(x, z0, z1)
    got = to_host(x)
    plan.close()
    ref = O.mpa_propagate(a, dt, dmm, L, M, nit, z0, z1)
    assert rel_l2(got, ref) < TOL[prec]


def test_blocking_error_at_2_16_modes():
    """FP64 blocked (B = 4096, H = 512) against FP64 full window on the
    2^16-mode 4-channel field over 40 long steps: the blocks change the
    channel band by less than 1e-7 (the roll-off removes only out-of-band
    content)."""
    import paper_1101_0086_amd as P
    n, dt = 1 << 16, 10.0 / 1024
    a = wdm_field(Grid(n, dt), 64, 4, "ook", np.random.default_rng(52))
    band = 65.0
    dmm = dm_map(beta3=0.1)
    L, M, nit = 2.5e-4, 2, 2
    out = {}
    for block, halo in ((0, 0), (4096, 512)):
        say("blocking error", block)
        plan = P.MPAPlan(n, dt, dmm, L, M, nit, block, halo, 1, band)
        x = to_dev(a, 1)
        plan.propagate(x, 0.0, 40 * L)
        out[block] = to_host(x)
        plan.close()
    omega = 2 * math.pi * np.fft.fftfreq(n, dt)
    inb = np.abs(omega) <= band + 50
    fb, ff = np.fft.fft(out[4096]), np.fft.fft(out[0])
    e_band = float(np.linalg.norm((fb - ff)[inb]) / np.linalg.norm(ff[inb]))
    assert e_band < 1e-7, e_band
    assert rel_l2(out[4096], out[0]) < 1e-4


def test_window_refusals():
    import torch
    import paper_1101_0086_amd as P
    dmm = dm_map()
    with pytest.raises(P.MPAError) as e:
        P.MPAPlan(1 << 23, 0.01, dmm, 0.05, 2, 2, 0, 0, 0)
    assert e.value.status == P._lib.MPA_EUNSUPPORTED
    with pytest.raises(P.MPAError):
        P.MPAPlan(1 << 14, 0.01, dmm, 0.05, 2, 2, 0, 0, 0, schedule=P.MPA_NODE_PARALLEL)
    plan = P.MPAPlan(1 << 14, 0.01, dmm, 0.05, 2, 2, 0, 0, 1)
    x = torch.zeros(1 << 14, dtype=torch.complex128, device="cuda:0")
    ck = plan.propagate_checkpointed(x, 0.0, 0.1)
    with pytest.raises(P.MPAError) as e:
        plan.adjoint(ck, x.clone(), 0.0, 0.1)
    assert e.value.status == P._lib.MPA_EUNSUPPORTED
