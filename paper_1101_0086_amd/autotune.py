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
signal band within the halo rule; the tuner times a few launches of each on
the GPU and keeps the cheapest per unit distance.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

BLOCKS = (512, 1024, 2048, 4096)
HALO_FRACTIONS = ((1, 8), (1, 4), (3, 8))   # halo B/8, B/4, 3B/8: overlap 2H/B of 25, 50, 75 %
HALO_RULE = 0.25          # the library's check: rate * L <= 0.25 * halo * dt


@dataclasses.dataclass
class Candidate:
    block: int
    halo: int
    L: float
    M: int
    seconds_per_unit_z: Optional[float] = None


def _steps(length: float, h: float) -> int:
    k = int(round(length / h))
    if k < 1 or abs(k * h - length) > 1e-9 * max(length, h):
        raise ValueError(f"dz = {h} does not divide {length}")
    return k


def candidates(n: int, dt: float, dmmap, dz: float, omega_band: float,
               blocks=BLOCKS, halo_fractions=HALO_FRACTIONS) -> List[Candidate]:
    """One candidate per block size B <= n and halo B p/q ((p, q) in halo_fractions):
    the longest long step that is a multiple of dz, divides every span (and
    the amplifier spacing) and satisfies the halo rule for every span."""
    counts = [_steps(s, dz) for s in dmmap.seg_len]
    if dmmap.z_amp > 0:
        counts.append(_steps(dmmap.z_amp, dz))
    g = 0
    for c in counts:
        g = math.gcd(g, c)
    rate = max(abs(b2) * omega_band + 0.5 * abs(b3) * omega_band ** 2
               for b2, b3 in zip(dmmap.beta2, dmmap.beta3))
    out = []
    for B in blocks:
        if B > n:
            continue
        for num, den in halo_fractions:
            H = B * num // den
            lmax = HALO_RULE * H * dt / rate if rate > 0 else float("inf")
            best = 0
            for k in range(1, g + 1):
                if g % k == 0 and k * dz <= lmax * (1 - 1e-12):
                    best = k
            if best:
                out.append(Candidate(B, H, best * dz, best))
    return out


def autotune(field, dt: float, dmmap, dz: float, n_iter: int, omega_band: float,
             precision: int = 0, launches: int = 40, blocks=BLOCKS, halo_fractions=HALO_FRACTIONS):
    """Time every candidate on `field` (a complex CUDA tensor, left
    unchanged) and return (best Candidate, list of all timed candidates)."""
    import torch

    from . import MPAPlan

    n = field.numel()
    cands = candidates(n, dt, dmmap, dz, omega_band, blocks, halo_fractions)
    if not cands:
        raise ValueError("no block size satisfies the halo rule at this dz")
    for c in cands:
        plan = MPAPlan(n, dt, dmmap, c.L, c.M, n_iter, c.block, c.halo, precision, omega_band)
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
                  precision: int = 0, tol: float = 1e-5, steps: int = 200, max_iter: int = 5):
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
        plan = MPAPlan(n, dt, dmmap, L, M, nit, block, halo, precision, omega_band)
        x = field.clone()
        plan.propagate(x, 0.0, steps * L)
        plan.close()
        outs[nit] = x
    ref = outs[max_iter]
    norm = float(torch.linalg.vector_norm(ref))
    dist = {nit: float(torch.linalg.vector_norm(outs[nit] - ref)) / norm for nit in outs}
    best = next(nit for nit in sorted(dist) if dist[nit] <= tol)
    return best, dist
