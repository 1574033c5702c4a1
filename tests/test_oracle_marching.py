"""Oracle pins: time blocking, marching, lumped gain, resume.

* One block covering the window reproduces the full-window MPA bitwise.
* Shifting the input by a whole number of block cores shifts the blocked
  output by the same amount (no hidden dependence on the block index).
* With sigma = 0 the blocked MPA equals exact linear propagation to within a
  small error once the halo exceeds the group-delay excursion of the signal
  over the long step, and fails clearly when it does not; the blocked linear
  map never grows the norm of broadband input (the spectral roll-off).
* Marching is memoryless: propagate(z0 -> z1 -> z2) equals propagate(z0 -> z2).
* A global phase factor commutes with the method.
* The lumped gain exp(gamma z_a) exactly undoes one amplifier span of loss.
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import Grid, dm_map, wdm_field


def _field(n=4096, dt=10 / 256, bits=16, ch=1, seed=1):
    return wdm_field(Grid(n, dt), bits, ch, "ook", np.random.default_rng(seed))


def test_single_block_is_full_window_bitwise():
    a = _field()
    dt = 10 / 256
    args = (20.0, 0.0, 1.0, 0.05, 0.05, 8, 3)
    full = O.mpa_long_step(a, O.omega_grid(a.size, dt), *args)
    blk = O.mpa_blocked_long_step(a, dt, a.size, 0, *args)
    assert np.array_equal(full, blk)


def test_block_partition_covers_each_sample_once():
    for n, b, h in ((4096, 1024, 128), (1 << 14, 4096, 512), (5000, 512, 64)):
        parts = O.block_partition(n, b, h)
        owned = np.zeros(n, int)
        for w0, c0, clen in parts:
            assert w0 == c0 - h and 0 < clen <= b - 2 * h
            owned[c0:c0 + clen] += 1
        assert np.all(owned == 1)


def test_blocked_shift_equivariance():
    n, dt, B, H = 8192, 10 / 512, 1024, 128
    C = B - 2 * H
    a = wdm_field(Grid(n, dt), 16, 2, "ook", np.random.default_rng(2))
    args = (dt, B, H, 20.0, 0.1, 1.0, 0.05, 2e-3, 4, 2)
    out = O.mpa_blocked_long_step(a, *args)
    shift = 3 * C
    # n is not a multiple of C: only shifts keeping the partition aligned are
    # exact, which holds for samples whose block does not wrap
    out_s = O.mpa_blocked_long_step(np.roll(a, shift), *args)
    nb_full = n // C
    lo, hi = shift, nb_full * C
    assert np.max(np.abs(out_s[lo:hi] - np.roll(out, shift)[lo:hi])) == 0.0


def test_block_taper_shape():
    w = O.block_taper(4096, 512)
    assert np.all(w[256:4096 - 256] == 1.0)
    assert np.array_equal(w[:256], w[::-1][:256])
    assert w[0] < 1e-8 and 1 - w[255] < 1e-8 and np.all(np.diff(w[:256]) > 0)
    assert np.all(O.block_taper(1024, 0) == 1.0)


def test_blocked_linear_error_controlled_by_halo():
    """sigma = 0: the tapered blocks reproduce exact linear propagation once
    the group delay of the signal band over L stays well inside the halo,
    and fail clearly when it does not."""
    n, dt, B, H = 8192, 10 / 512, 1024, 128
    a = wdm_field(Grid(n, dt), 32, 3, "ook", np.random.default_rng(4))
    b2 = 20.0
    rate = O.halo_rate(45.0, b2, 0.0)
    for frac, good in ((0.1, True), (0.2, True), (1.5, False)):
        L = frac * H * dt / rate
        exact = O.linear_step(a, O.omega_grid(n, dt), b2, 0.0, 0.0, L)
        out = O.mpa_blocked_long_step(a, dt, B, H, b2, 0.0, 0.0, 0.0, L, 2, 1)
        err = O.rel_l2(out, exact)
        assert (err < 1e-9) if good else (err > 1e-3)


def test_block_mask_shape():
    B, H, dt = 4096, 512, 10 / 1024
    om = O.omega_grid(B, dt)
    rate = O.halo_rate(145.0, 20.0, 0.1)
    L = 0.25 * H * dt / rate
    m = O.block_mask(om, 20.0, 0.1, L, H, dt)
    assert np.all((m >= 0) & (m <= 1))
    assert np.all(m[np.abs(om) <= 145.0] == 1.0)          # the halo rule's band passes
    assert np.all(m[np.abs(om) >= 0.9 * math.pi / dt] == 0.0)
    g = np.abs(20.0 * om + 0.05 * om ** 2) * L / (H * dt)
    assert np.all(m[g >= 0.5] == 0.0)


def test_blocked_linear_map_is_stable():
    """Stitching overlapping periodic windows is not unitary: without the
    spectral roll-off, broadband content at the Nyquist wrap grows by a few
    percent per long step when beta3 != 0.  With it the norm never grows."""
    n, dt, B, H = 8192, 10 / 1024, 2048, 256
    rng = np.random.default_rng(0)
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    L = 0.5 / 8000
    x = O.mpa_blocked_long_step(x, dt, B, H, 20.0, 0.1, 0.0, 0.0, L, 1, 1)
    n0 = np.linalg.norm(x)
    for m in range(600):
        x = O.mpa_blocked_long_step(x, dt, B, H, 20.0 if m < 300 else -19.8, 0.1, 0.0, 0.0, L, 1, 1)
    assert np.linalg.norm(x) <= n0 * (1 + 1e-9)


def test_blocked_nonlinear_close_to_full_window():
    """The blocking error of the full method (8 channels, beta3 != 0, loss)
    over many long steps, on the channels' band (the roll-off removes only
    four-wave-mixing products beyond it, which this grid would alias)."""
    n, dt, B, H = 1 << 13, 10 / 1024, 2048, 256
    a = wdm_field(Grid(n, dt), 8, 8, "ook", np.random.default_rng(7))
    rate = O.halo_rate(145.0, 20.0, 0.1)
    L = 0.5 / math.ceil(0.5 / (0.25 * H * dt / rate))
    dmm = dm_map(beta3=0.1)
    x, y = a.copy(), a.copy()
    for m in range(60):
        x = O.mpa_step(x, dt, dmm, L, 2, 2, m, B, H)
        y = O.mpa_step(y, dt, dmm, L, 2, 2, m)
    om = O.omega_grid(n, dt)

    def band(v):
        s = O.paper_fft(v)
        s[np.abs(om) > 200.0] = 0
        return s

    assert O.rel_l2(band(x), band(y)) < 1e-7
    assert O.rel_l2(x, y) < 1e-4


def test_marching_resume_and_global_phase():
    a = _field()
    dt = 10 / 256
    dmm = dm_map(beta3=0.0)
    L, M, nit = 0.05, 4, 2
    whole = O.mpa_propagate(a, dt, dmm, L, M, nit, 0.0, 1.5)
    part = O.mpa_propagate(a, dt, dmm, L, M, nit, 0.0, 0.75)
    part = O.mpa_propagate(part, dt, dmm, L, M, nit, 0.75, 1.5)
    assert np.array_equal(whole, part)
    ph = np.exp(0.7j)
    rot = O.mpa_propagate(a * ph, dt, dmm, L, M, nit, 0.0, 0.25)
    assert O.rel_l2(rot, ph * O.mpa_propagate(a, dt, dmm, L, M, nit, 0.0, 0.25)) < 1e-14


def test_lumped_gain_restores_span_loss():
    a = _field()
    dt = 10 / 256
    dmm = O.DMMapSpec((0.5, 0.5), (0.0, 0.0), (0.0, 0.0), (0.0, 0.0), 0.3, 1.0)
    out = O.mpa_propagate(a, dt, dmm, 0.1, 2, 1, 0.0, 1.0)
    assert O.rel_l2(out, a) < 1e-14
    half = O.mpa_propagate(a, dt, dmm, 0.1, 2, 1, 0.0, 0.5)
    assert O.rel_l2(half, a * math.exp(-0.3 * 0.5)) < 1e-14
    ss = O.ss_propagate(a, dt, dmm, 0.05, 0.0, 1.0)
    assert O.rel_l2(ss, a) < 1e-14


def test_span_schedule_uses_integer_counters():
    dmm = dm_map()
    L = 0.1
    spans = [O.span_of_long_step(dmm, L, m) for m in range(20)]
    assert spans == ([0] * 5 + [1] * 5) * 2
    with pytest.raises(ValueError):
        O.span_of_long_step(dmm, 0.3, 0)


# ---- window shift (windows moved against their cores) ----------------------

def _one_sided():
    """Three channels (band 45) with beta3 = 2: the group-delay rate
    20 omega + omega^2 over the band runs from -100 to 2925, mostly one-signed.
    Halo of 10 time units (pulse width 1), so that the taper's own
    broadening of the content it touches stays far from the core."""
    n, dt, B, H = 8192, 10 / 512, 2048, 512
    a = wdm_field(Grid(n, dt), 32, 3, "ook", np.random.default_rng(4))
    return n, dt, B, H, a, 45.0, 20.0, 2.0


def test_group_delay_range_and_excursion():
    lo, hi = O.group_delay_range(45.0, 20.0, 2.0)
    om = np.linspace(-45.0, 45.0, 200001)
    u = 20.0 * om + om ** 2
    assert abs(lo - u.min()) < 1e-6 and abs(hi - u.max()) < 1e-6
    assert O.group_delay_range(145.0, 20.0, 0.0) == (-2900.0, 2900.0)
    L, dt, s = 3e-4, 0.01, 40
    assert abs(O.halo_excursion(45.0, 20.0, 2.0, L, s, dt) - np.max(np.abs(u * L - s * dt))) < 1e-9


def test_block_partition_with_shift():
    for n, b, h, s in ((4096, 1024, 128, 37), (1 << 14, 4096, 512, -200), (5000, 512, 64, 32)):
        owned = np.zeros(n, int)
        for w0, c0, clen in O.block_partition(n, b, h, s):
            assert w0 == c0 - h - s and 0 < clen <= b - 2 * h
            owned[c0:c0 + clen] += 1
        assert np.all(owned == 1)


def test_window_shift_centres_the_domain_of_dependence():
    """sigma = 0 with a one-sided group delay: a long step whose band
    excursion is a quarter of the halo only once the window is shifted by the
    middle of the group-delay range reproduces exact linear propagation;
    unshifted, or shifted the wrong way, the content reaches the tapered
    outer halo and the blocked result fails."""
    n, dt, B, H, a, band, b2, b3 = _one_sided()
    lo, hi = O.group_delay_range(band, b2, b3)
    L = 0.25 * H * dt / (0.5 * (hi - lo))
    s = int(round(0.5 * (lo + hi) * L / dt))
    assert 0 < s <= H // 2
    assert O.halo_excursion(band, b2, b3, L, s, dt) <= 0.25 * H * dt * 1.01
    exact = O.linear_step(a, O.omega_grid(n, dt), b2, b3, 0.0, L)
    errs = {}
    for shift in (s, 0, -s):
        out = O.mpa_blocked_long_step(a, dt, B, H, b2, b3, 0.0, 0.0, L, 2, 1, shift=shift)
        errs[shift] = O.rel_l2(out, exact)
    assert errs[s] < 1e-9, errs
    assert errs[0] > 1e-2 and errs[-s] > 1e-1, errs
    with pytest.raises(ValueError):
        O.mpa_blocked_long_step(a, dt, B, H, b2, b3, 0.0, 0.0, L, 2, 1, shift=H // 2 + 1)


def test_window_shift_equivariance_and_mask():
    n, dt, B, H = 8192, 10 / 512, 1024, 128
    C = B - 2 * H
    a = wdm_field(Grid(n, dt), 16, 2, "ook", np.random.default_rng(2))
    kw = dict(shift=23)
    args = (dt, B, H, 20.0, 0.1, 1.0, 0.05, 2e-3, 4, 2)
    out = O.mpa_blocked_long_step(a, *args, **kw)
    out_s = O.mpa_blocked_long_step(np.roll(a, 3 * C), *args, **kw)
    lo, hi = 3 * C, (n // C) * C
    assert np.max(np.abs(out_s[lo:hi] - np.roll(out, 3 * C)[lo:hi])) == 0.0
    # the roll-off passes the band once the shifted excursion obeys the halo rule
    band, b2, b3 = 45.0, 20.0, 2.0
    glo, ghi = O.group_delay_range(band, b2, b3)
    L = 0.25 * H * dt / (0.5 * (ghi - glo))
    s = int(round(0.5 * (glo + ghi) * L / dt))
    om = O.omega_grid(B, dt)
    m = O.block_mask(om, b2, b3, L, H, dt, s)
    assert np.all(m[np.abs(om) <= band] == 1.0)
    g = np.abs((b2 * om + 0.5 * b3 * om ** 2) * L - s * dt) / (H * dt)
    assert np.all(m[g >= 0.5] == 0.0) and np.all(m[(g <= 0.35) & (np.abs(om) * dt / math.pi <= 0.8)] == 1.0)
