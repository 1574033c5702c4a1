"""The seeded synthetic inputs: deterministic, power-normalised, carriers on
the grid, and the fast slot-wise builder equal to the direct one."""
import math

import numpy as np

from workloads import Grid, WORKLOADS, wdm_field
from workloads.wdm import _fast_wdm_field


def test_seeded_and_normalised():
    g = Grid(4096, 10 / 256)
    a = wdm_field(g, 16, 1, "ook", np.random.default_rng(1))
    b = wdm_field(g, 16, 1, "ook", np.random.default_rng(1))
    assert np.array_equal(a, b)
    assert abs(np.mean(np.abs(a) ** 2) - 1 / 20) < 1e-12


def test_fast_builder_matches_direct():
    g = Grid(1 << 13, 10 / 1024)
    for mod in ("ook", "qpsk"):
        a = wdm_field(g, 8, 3, mod, np.random.default_rng(5))
        b = _fast_wdm_field(g, 8, 3, mod, np.random.default_rng(5))
        assert np.max(np.abs(a - b)) < 1e-12


def test_channel_spectra_on_grid_and_in_band():
    w = WORKLOADS["wdm8_n262144_f32"]
    g = Grid(1 << 14, w.grid.dt)
    a = wdm_field(g, 16, 8, "ook", np.random.default_rng(2))
    spec = np.abs(np.fft.ifft(a)) ** 2
    omega = 2 * math.pi * np.fft.fftfreq(g.n, g.dt)
    out_band = spec[np.abs(omega) > w.omega_sig].sum() / spec.sum()
    assert out_band < 1e-9


def test_workload_geometry_is_consistent():
    for w in WORKLOADS.values():
        s = w.mpa
        for seg in w.dmmap.seg_len:
            assert abs(round(seg / s.L) * s.L - seg) < 1e-12
        if s.block:
            assert s.block > 2 * s.halo and w.grid.n % 2 == 0 and abs(s.shift) <= s.halo // 2
            # group-delay rate over the band, relative to the window shift (both spans)
            for b2, b3 in zip(w.dmmap.beta2, w.dmmap.beta3):
                om = np.linspace(-s.omega_band, s.omega_band, 20001)
                u = b2 * om + 0.5 * b3 * om ** 2
                assert np.max(np.abs(u * s.L - s.shift * w.grid.dt)) <= 0.25 * s.halo * w.grid.dt
