"""MPA on windows larger than one workgroup's transform (four-step
transforms, 8192 <= N <= 2^22) through the C ABI: the full window against the
FP64 oracle's full-window MPA (no blocks) at sizes the oracle runs in
seconds, across a span change and an amplifier, both precisions; time blocks
of 8192..32768 against the oracle's blocked MPA (taper, roll-off, shifted
windows, ragged last core); and the blocking error of the time-blocked plan
measured against the full window at 2^16 modes."""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import TOL_F32, TOL_F64, centred_shift, rel_l2, say, to_dev, to_host
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


def _large_block_case(n, H, seed):
    """WDM field (4 OOK channels, 128 samples per bit) and the longest L = 0.5/k
    within the halo rule for the 65-wide band."""
    dt = 10.0 / 1024
    a = wdm_field(Grid(n, dt), n // 128, 4, "ook", np.random.default_rng(seed))
    band = 65.0
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(0.5 / (0.25 * H * dt / rate))
    while (0.5 / k) * rate > 0.25 * H * dt:
        k += 1
    return a, dt, band, 0.5 / k


@pytest.mark.parametrize("n,B,H,prec,shifted", [
    (1 << 15, 8192, 1024, 1, False),
    (1 << 15, 8192, 1024, 0, False),
    (1 << 16, 16384, 3072, 0, True),
    (1 << 17, 32768, 4096, 1, True),
    # a block as long as the field, with halos: two windows wrapping around it
    (1 << 15, 32768, 4096, 1, True),
])
def test_blocks_above_4096_against_oracle(n, B, H, prec, shifted):
    """Blocked plans with B > 4096 (gather with halos and taper, roll-off,
    stitched cores; ragged last core) across the span change and, for the
    FP64 8192-blocks, an amplifier; also B = N with halos (the autotuner's
    largest candidate on a 2^15-mode field), whose windows wrap around the
    field."""
    import paper_1101_0086_amd as P
    a, dt, band, L = _large_block_case(n, H, 72)
    dmm = dm_map(beta3=0.1)
    sh = centred_shift(band, dmm, L, dt, H) if shifted else 0
    M, nit = 4, 2
    ranges = [(0.5 - 2 * L, 0.5 + 2 * L)]
    if B == 8192 and prec == 1:
        ranges.append((1.0 - 2 * L, 1.0 + L))
    plan = P.MPAPlan(n, dt, dmm, L, M, nit, B, H, prec, band, shift=sh)
    assert plan.info()["n_blocks"] == -(-n // (B - 2 * H))
    assert n % (B - 2 * H) != 0                       # the last core is ragged
    for z0, z1 in ranges:
        say("large blocks", n, B, H, prec, sh, z0, z1)
        x = to_dev(a, prec)
        plan.propagate(x, z0, z1)
        ref = O.mpa_propagate(a, dt, dmm, L, M, nit, z0, z1, B, H, sh)
        assert rel_l2(to_host(x), ref) < TOL[prec], (z0, z1)
    plan.close()


def test_large_blocks_refusals():
    """Blocks above 4096 run in node order only, with no reverse pass and no
    batches; blocks above 2^22 are refused (L = 0.005 and a band of 10 keep
    the halo rule)."""
    import torch
    import paper_1101_0086_amd as P
    dmm = dm_map()
    L, band = 0.005, 10.0
    with pytest.raises(P.MPAError) as e:
        P.MPAPlan(1 << 16, 0.01, dmm, L, 2, 2, 8192, 1024, 0, band, schedule=P.MPA_NODE_PARALLEL)
    assert e.value.status == P._lib.MPA_EUNSUPPORTED
    with pytest.raises(P.MPAError) as e:
        P.MPABatchPlan([1 << 15, 1 << 14], 0.01, dmm, L, 2, 2, 8192, 1024, P.MPA_C64, band)
    assert e.value.status == P._lib.MPA_EUNSUPPORTED
    with pytest.raises(P.MPAError) as e:
        P.MPAPlan(1 << 24, 0.01, dmm, L, 2, 2, 1 << 23, 1024, 0, band)
    assert e.value.status == P._lib.MPA_EUNSUPPORTED
    plan = P.MPAPlan(1 << 15, 0.01, dmm, L, 2, 2, 8192, 1024, 1, band)
    x = torch.zeros(1 << 15, dtype=torch.complex128, device="cuda:0")
    ck = plan.propagate_checkpointed(x, 0.0, 0.1)
    with pytest.raises(P.MPAError) as e:
        plan.adjoint(ck, x.clone(), 0.0, 0.1)
    assert e.value.status == P._lib.MPA_EUNSUPPORTED
    plan.close()


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


@pytest.mark.parametrize("prec", [1, 0])
def test_large_blocks_with_crossing_steps_and_distributed_gain(prec):
    """8192-blocks with L = 1/k, k odd (steps across the span boundary at 0.5
    and 1.5, sigma 1 and 2) and distributed gain, over an amplifier: the
    window path takes the boundary-crossing tables and the combined gain rows
    of the fused path."""
    import paper_1101_0086_amd as P
    from workloads.wdm import DMMap
    n, B, H = 1 << 15, 8192, 1024
    a, dt, band, _ = _large_block_case(n, H, 74)
    rate = O.halo_rate(band, 20.0, 0.1)
    k = math.ceil(1.0 / (0.25 * H * dt / rate))
    k += 1 - k % 2                                   # odd: L divides the period, not the spans
    L = 1.0 / k
    base = dm_map(beta3=0.1)
    dmm = DMMap(**{**base.__dict__, "sigma": (1.0, 2.0), "raman_g0": 0.2, "raman_alpha": 3.0})
    m0 = k // 2 - 2
    z0, z1 = m0 * L, (m0 + 5) * L
    for zz0, zz1 in ((z0, z1), (1.0 - 2 * L, 1.0 + 2 * L)):
        say("large blocks, crossing steps, gain", prec, zz0, zz1)
        plan = P.MPAPlan(n, dt, dmm, L, 3, 2, B, H, prec, band)
        x = to_dev(a, prec)
        plan.propagate(x, zz0, zz1)
        plan.close()
        ref = O.mpa_propagate(a, dt, dmm, L, 3, 2, zz0, zz1, B, H)
        assert rel_l2(to_host(x), ref) < TOL[prec], (zz0, zz1)
