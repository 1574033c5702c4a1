"""Synthetic dispersion-managed WDM workloads (seeded).

The paper's own system parameters live in an earlier letter that this
project does not have, so its experiments (five, three and twenty channel
WDM links over DM fibre) are stood in for by the synthetic workloads below.
Each is a pseudo-random train of Gaussian return-to-zero pulses per channel,
on a periodic time grid, over a two-span dispersion map:

* bit slot ``T_b = 10`` time units, pulse ``p exp(-t^2 / (2 tau^2))`` with
  ``tau = 0.1 T_b`` (one pulse per slot, centred in the slot);
* channel carriers ``exp(-i Omega_c t)`` with ``Omega_c`` spaced by 40 and
  centred on zero, snapped to the grid's frequency spacing ``2 pi / T``;
* on-off keying (bit in {0, 1}) or QPSK (``exp(i (pi/4 + k pi/2))``, every
  slot filled);
* the whole field is scaled so that ``mean |A|^2 = 1 / (20 sigma)``, i.e. the
  average-power nonlinear length is 20 DM periods;
* the map alternates spans of length 0.5 with beta2 = +20 and beta2 = -19.8,
  loss gamma = 0.05 and a lumped amplifier at every integer z.

Nothing here evaluates the NLSE or any step of the propagation method.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

T_BIT = 10.0          # bit slot, time units
TAU = 0.1 * T_BIT     # Gaussian 1/e half-width of |A|^2 ... of exp(-t^2/2tau^2)
CHANNEL_SPACING = 40.0


@dataclasses.dataclass(frozen=True)
class DMMap:
    """One period of a piecewise-constant dispersion map.

    ``seg_len[i]``, ``beta2[i]``, ``beta3[i]``, ``sigma[i]`` hold span ``i``;
    ``gamma`` is the amplitude loss rate and ``z_amp`` the amplifier spacing
    (0 disables amplifiers); ``raman_g0``, ``raman_alpha`` add a distributed
    gain g0 exp(-alpha (z_a - zeta)) at position zeta of each amplifier
    period.  The period is ``sum(seg_len)``.
    """
    seg_len: tuple
    beta2: tuple
    beta3: tuple
    sigma: tuple
    gamma: float = 0.0
    z_amp: float = 0.0
    raman_g0: float = 0.0       # distributed gain g0 exp(-alpha (z_a - zeta)) (0: none)
    raman_alpha: float = 0.0

    @property
    def period(self) -> float:
        return float(sum(self.seg_len))

    def with_sigma(self, sigma: float) -> "DMMap":
        return dataclasses.replace(self, sigma=tuple(float(sigma) for _ in self.seg_len))


def dm_map(beta3: float = 0.0, sigma: float = 1.0, gamma: float = 0.05,
           z_amp: float = 1.0, beta2=(20.0, -19.8), seg=(0.5, 0.5)) -> DMMap:
    """The two-span map of the workloads (+20 first, then -19.8)."""
    return DMMap(seg_len=tuple(float(s) for s in seg),
                 beta2=tuple(float(b) for b in beta2),
                 beta3=tuple(float(beta3) for _ in seg),
                 sigma=tuple(float(sigma) for _ in seg),
                 gamma=float(gamma), z_amp=float(z_amp))


@dataclasses.dataclass(frozen=True)
class Grid:
    n: int        # number of time samples (= number of Fourier harmonics)
    dt: float     # sample spacing; the periodic window is n * dt

    @property
    def window(self) -> float:
        return self.n * self.dt


@dataclasses.dataclass(frozen=True)
class MPASettings:
    """Long step L, M quadrature intervals per long step, n_iter Picard sweeps,
    time blocks of ``block`` points with ``halo`` points of overlap per side
    (``block = 0`` means one block covering the whole window), windows moved
    ``shift`` samples against their cores."""
    L: float
    M: int
    n_iter: int
    block: int = 0
    halo: int = 0
    omega_band: float = 0.0   # highest |omega| carrying signal (halo rule); 0 = grid edge
    shift: int = 0


def _periodic_offsets(t: np.ndarray, centre: float, window: float) -> np.ndarray:
    """Minimum-image distance on the periodic window (other images of a
    tau = 1 pulse lie at least window/2 >= 80 away and are below 1e-300)."""
    d = (t - centre + 0.5 * window) % window - 0.5 * window
    return d


def wdm_field(grid: Grid, n_bits: int, n_channels: int, modulation: str,
              rng: np.random.Generator, sigma: float = 1.0,
              mean_power: Optional[float] = None) -> np.ndarray:
    """Complex128 field A(t_n, 0), t_n = n dt, for ``n_channels`` WDM channels.

    Draw order (fixed, so that a seed pins the field): for each channel, its
    ``n_bits`` symbols.  ``mean_power`` defaults to 1 / (20 sigma).
    """
    n, dt = grid.n, grid.dt
    window = n * dt
    t = dt * np.arange(n)
    t_bit = window / n_bits
    dw = 2.0 * math.pi / window
    field = np.zeros(n, dtype=np.complex128)
    for c in range(n_channels):
        omega_c = (c - 0.5 * (n_channels - 1)) * CHANNEL_SPACING
        omega_c = dw * round(omega_c / dw)
        if modulation == "ook":
            sym = rng.integers(0, 2, size=n_bits).astype(np.complex128)
        elif modulation == "qpsk":
            k = rng.integers(0, 4, size=n_bits)
            sym = np.exp(1j * (math.pi / 4 + k * math.pi / 2))
        else:
            raise ValueError(f"unknown modulation {modulation!r}")
        env = np.zeros(n, dtype=np.complex128)
        for b in range(n_bits):
            if sym[b] == 0:
                continue
            d = _periodic_offsets(t, (b + 0.5) * t_bit, window)
            env += sym[b] * np.exp(-d * d / (2.0 * TAU * TAU))
        field += env * np.exp(-1j * omega_c * t)
    p = 1.0 / (20.0 * sigma) if mean_power is None else mean_power
    cur = float(np.mean(np.abs(field) ** 2))
    if cur > 0:
        field *= math.sqrt(p / cur)
    return field


def _fast_wdm_field(grid: Grid, n_bits: int, n_channels: int, modulation: str,
                    rng: np.random.Generator, sigma: float = 1.0) -> np.ndarray:
    """Same field as :func:`wdm_field` (same draws, same samples up to
    rounding) for the large grids: each channel's envelope is the circular
    convolution of its symbol comb (one symbol every slot) with the pulse of
    slot 0, and its carrier (a whole number q of grid frequencies) is a
    shift of that spectrum by q bins; one inverse FFT builds the field."""
    n, dt = grid.n, grid.dt
    window = n * dt
    t_bit = window / n_bits
    spb = n // n_bits                 # samples per bit slot (exact for all workloads)
    assert spb * n_bits == n
    dw = 2.0 * math.pi / window
    t = dt * np.arange(n)
    d0 = _periodic_offsets(t, 0.5 * t_bit, window)
    g_hat = np.fft.fft(np.exp(-d0 * d0 / (2.0 * TAU * TAU)))
    spec = np.zeros(n, dtype=np.complex128)
    for c in range(n_channels):
        q = int(round((c - 0.5 * (n_channels - 1)) * CHANNEL_SPACING / dw))
        if modulation == "ook":
            sym = rng.integers(0, 2, size=n_bits).astype(np.complex128)
        else:
            k = rng.integers(0, 4, size=n_bits)
            sym = np.exp(1j * (math.pi / 4 + k * math.pi / 2))
        # comb spectrum: the symbols' n_bits-point DFT repeated spb times
        comb_hat = np.tile(np.fft.fft(sym), spb)
        # exp(-i q dw t) shifts numpy's spectrum down by q bins
        spec += np.roll(comb_hat * g_hat, -q)
    field = np.fft.ifft(spec)
    p = 1.0 / (20.0 * sigma)
    cur = float(np.mean(np.abs(field) ** 2))
    if cur > 0:
        field *= math.sqrt(p / cur)
    return field


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    grid: Grid
    n_bits: int
    n_channels: int
    modulation: str
    dmmap: DMMap
    periods: int
    mpa: MPASettings
    precision: str          # "f64" or "f32" (field and FFTs; phases are FP64-built)
    seed: int
    omega_sig: float        # highest |omega| with signal content

    def field(self, seed: Optional[int] = None) -> np.ndarray:
        rng = np.random.default_rng(self.seed if seed is None else seed)
        sigma = self.dmmap.sigma[0]
        if self.grid.n <= 1 << 14:
            return wdm_field(self.grid, self.n_bits, self.n_channels,
                             self.modulation, rng, sigma)
        return _fast_wdm_field(self.grid, self.n_bits, self.n_channels,
                               self.modulation, rng, sigma)


def _omega_sig(n_channels: int) -> float:
    return 0.5 * (n_channels - 1) * CHANNEL_SPACING + 5.0


WORKLOADS = {
    # small case: FP64, one 4096-point window, single OOK channel
    "dm1ch_n4096_f64": Workload(
        "dm1ch_n4096_f64", Grid(1 << 12, T_BIT / 256), 16, 1, "ook",
        dm_map(beta3=0.0), 10, MPASettings(L=0.05, M=16, n_iter=3),
        "f64", 1, _omega_sig(1)),
    # 8-channel WDM, 2^18 modes, FP32 field with FP64 phases, 4096-blocks 25% overlap
    "wdm8_n262144_f32": Workload(
        "wdm8_n262144_f32", Grid(1 << 18, T_BIT / 1024), 256, 8, "ook",
        dm_map(beta3=0.1), 100,
        MPASettings(L=2.5e-4, M=4, n_iter=2, block=4096, halo=512,
                    omega_band=_omega_sig(8)),
        "f32", 2, _omega_sig(8)),
    # 32-channel QPSK WDM, 2^22 modes; dz = 7.8125e-6, block size, overlap and
    # window shift as the autotuner picks them at that dz (4096-blocks, 1024-halo,
    # four dz per long step, windows moved 192 samples against their cores)
    "wdm32_n4194304_f32": Workload(
        "wdm32_n4194304_f32", Grid(1 << 22, T_BIT / 4096), 1024, 32, "qpsk",
        dm_map(beta3=0.1), 200,
        MPASettings(L=3.125e-5, M=4, n_iter=2, block=4096, halo=1024,
                    omega_band=_omega_sig(32), shift=192),
        "f32", 3, _omega_sig(32)),
    # 4-channel, 2^16 modes (the gradient workload's forward)
    "wdm4_n65536_f32": Workload(
        "wdm4_n65536_f32", Grid(1 << 16, T_BIT / 1024), 64, 4, "ook",
        dm_map(beta3=0.1), 20,
        MPASettings(L=2.5e-4, M=2, n_iter=2, block=2048, halo=256,
                    omega_band=_omega_sig(4)),
        "f32", 5, _omega_sig(4)),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def batched_instances(count: int = 256, seed: int = 4):
    """Instances of the batched workload: N uniform over 2^14..2^18, 1-16
    channels, OOK, sigma uniform in [0.5, 2].  Draw order per instance: N,
    channel count, sigma, then the channel bits.  Returns a list of
    (grid, n_channels, sigma, field)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = 1 << int(rng.integers(14, 19))
        nch = int(rng.integers(1, 17))
        sigma = float(rng.uniform(0.5, 2.0))
        grid = Grid(n, T_BIT / 2048)
        n_bits = n // 2048
        f = _fast_wdm_field(grid, n_bits, nch, "ook", rng, sigma)
        out.append((grid, nch, sigma, f))
    return out
