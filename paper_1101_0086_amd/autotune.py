"""Choice of block size, overlap, long step and nodes per long step at fixed
accuracy.

The leading error terms of both the MPA and split-step (Eqs. 5 and 7) are
L^3/M^2 per long step, i.e. (L/M)^2 = dz^2 per unit distance, so at a fixed
quadrature interval dz the accuracy is fixed and only the cost changes with
(B, H, L, M): larger blocks allow longer long steps (fewer of the three extra
transforms per long step) but cost more per point and give fewer blocks to
spread over the GPU; a wider halo H (overlap 2H/B of 25 %, 50 % or 75 %)
also allows a longer long step and gives more blocks (core B - 2H), at the
price of computing more samples twice.  For every compiled block size B and
halo B/8, B/4 or 3B/8 the candidate takes the longest long step L = k dz that divides
every span and the amplifier spacing and keeps the group delay of the
signal band within the halo rule, with the windows shifted against their
cores by the middle of the band's group-delay range over L (with beta3 != 0
the group delay is one-signed over much of a wide band, and the shift
centres the core's domain of dependence in its window); the tuner times a
few launches of each on the GPU and keeps the cheapest per unit distance.
Blocks of 512..4096 run in the fused long-step kernel; blocks of
8192..32768 run by four-step transforms in node order (every window's state
in HBM), which allows long steps up to 8 times longer at the same overlap.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

BLOCKS = (512, 1024, 2048, 4096, 8192, 16384, 32768)
HALO_FRACTIONS = ((1, 8), (1, 4), (3, 8))   # halo B/8, B/4, 3B/8: overlap 2H/B of 25, 50, 75 %
HALO_RULE = 0.25          # the library's check: rate * L <= 0.25 * halo * dt


@dataclasses.dataclass
class Candidate:
    block: int
    halo: int
    L: float
    M: int
    shift: int = 0
    seconds_per_unit_z: Optional[float] = None


def group_delay_range(omega_band: float, beta2: float, beta3: float):
    """(min, max) of beta2 omega + beta3 omega^2 / 2 over |omega| <= omega_band."""
    w = float(omega_band)
    vals = [beta2 * w + 0.5 * beta3 * w * w, -beta2 * w + 0.5 * beta3 * w * w]
    if beta3 != 0 and abs(beta2 / beta3) <= w:
        vals.append(-0.5 * beta2 * beta2 / beta3)
    return min(vals), max(vals)


def window_shift(dmmap, omega_band: float, L: float, dt: float, halo: int) -> int:
    """The shift the library takes for MPA_SHIFT_AUTO: round(c L / dt), c the
    middle of the group-delay range over the band and every span, clamped to
    +-halo/2."""
    r = [group_delay_range(omega_band, b2, b3) for b2, b3 in zip(dmmap.beta2, dmmap.beta3)]
    lo, hi = min(x[0] for x in r), max(x[1] for x in r)
    c = round(0.5 * (lo + hi) * L / dt)
    return int(max(-(halo // 2), min(halo // 2, c)))


def _fits(dmmap, omega_band: float, L: float, dt: float, halo: int, shift: int) -> bool:
    for b2, b3 in zip(dmmap.beta2, dmmap.beta3):
        lo, hi = group_delay_range(omega_band, b2, b3)
        if max(abs(lo * L - shift * dt), abs(hi * L - shift * dt)) > HALO_RULE * halo * dt:
            return False
    return True


def _steps(length: float, h: float) -> int:
    k = int(round(length / h))
    if k < 1 or abs(k * h - length) > 1e-9 * max(length, h):
        raise ValueError(f"dz = {h} does not divide {length}")
    return k


def candidates(n: int, dt: float, dmmap, dz: float, omega_band: float,
               blocks=BLOCKS, halo_fractions=HALO_FRACTIONS, shifted: bool = True) -> List[Candidate]:
    """One candidate per block size B <= n and halo B p/q ((p, q) in halo_fractions):
    the longest long step that is a multiple of dz, divides every span (and
    the amplifier spacing) and satisfies the halo rule for every span, with
    the windows shifted by :func:`window_shift` (``shifted``) or not."""
    counts = [_steps(s, dz) for s in dmmap.seg_len]
    if dmmap.z_amp > 0:
        counts.append(_steps(dmmap.z_amp, dz))
    g = 0
    for c in counts:
        g = math.gcd(g, c)
    out = []
    for B in blocks:
        if B > n:
            continue
        for num, den in halo_fractions:
            H = B * num // den
            best, best_shift = 0, 0
            for k in range(1, g + 1):
                if g % k:
                    continue
                L = k * dz
                sh = window_shift(dmmap, omega_band, L, dt, H) if shifted else 0
                if _fits(dmmap, omega_band, L * (1 + 1e-12), dt, H, sh):
                    best, best_shift = k, sh
            if best:
                out.append(Candidate(B, H, best * dz, best, best_shift))
    return out


def autotune(field, dt: float, dmmap, dz: float, n_iter: int, omega_band: float,
             precision: int = 0, launches: int = 40, blocks=BLOCKS, halo_fractions=HALO_FRACTIONS,
             shifted: bool = True):
    """Time every candidate on `field` (a complex CUDA tensor, left
    unchanged) and return (best Candidate, list of all timed candidates)."""
    import torch

    from . import MPAPlan

    n = field.numel()
    cands = candidates(n, dt, dmmap, dz, omega_band, blocks, halo_fractions, shifted)
    if not cands:
        raise ValueError("no block size satisfies the halo rule at this dz")
    for c in cands:
        plan = MPAPlan(n, dt, dmmap, c.L, c.M, n_iter, c.block, c.halo, precision, omega_band, shift=c.shift)
        x = field.clone()
        plan.propagate(x, 0.0, 4 * c.L)                 # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.propagate(x, 0.0, launches * c.L)
        torch.cuda.synchronize()
        c.seconds_per_unit_z = (time.perf_counter() - t0) / (launches * c.L)
        plan.close()
    best = min(cands, key=lambda c: c.seconds_per_unit_z)
    return best, cands


def choose_n_iter(field, dt, dmmap, L: float, M: int, block: int, halo: int, omega_band: float,
                  precision: int = 0, tol: float = 1e-5, steps: int = 200, max_iter: int = 5, shift: int = 0):
    """Smallest number of Picard sweeps whose result after `steps` long steps
    from `field` (a complex CUDA tensor, left unchanged) is within `tol`
    (relative L2) of the result with `max_iter` sweeps.

    The sweeps converge to the fixed point of the discretised integral
    equation (Eq. 6); the paper bounds the distance after n sweeps by the
    floor (L / z_nl)^(n+1) (text after Eq. 7), which for weakly nonlinear
    links is far below the quadrature error, so one or two sweeps suffice.
    The distance is measured here on the actual field instead of estimated.
    Returns (n_iter, {n: relative distance to the max_iter result})."""
    import torch

    from . import MPAPlan

    n = field.numel()
    outs = {}
    for nit in range(1, max_iter + 1):
        plan = MPAPlan(n, dt, dmmap, L, M, nit, block, halo, precision, omega_band, shift=shift)
        x = field.clone()
        plan.propagate(x, 0.0, steps * L)
        plan.close()
        outs[nit] = x
    ref = outs[max_iter]
    norm = float(torch.linalg.vector_norm(ref))
    dist = {nit: float(torch.linalg.vector_norm(outs[nit] - ref)) / norm for nit in outs}
    best = next(nit for nit in sorted(dist) if dist[nit] <= tol)
    return best, dist
