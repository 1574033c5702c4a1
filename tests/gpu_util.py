"""Helpers for the GPU tests: device transfer and the FP64/FP32 tolerances.

Tolerances (relative L2 over the whole field against the FP64 oracle on the
same input): 1e-10 for the FP64 path and 1e-5 for the FP32 path, on runs
short enough that FP32 rounding (about 3e-7 per long step, growing like the
square root of the number of long steps) stays below 1e-5.
"""
import sys

import numpy as np

TOL_F64 = 1e-10
TOL_F32 = 1e-5


def torch_mod():
    import torch
    return torch


def to_dev(a: np.ndarray, precision: int):
    torch = torch_mod()
    dt = torch.complex64 if precision == 0 else torch.complex128
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dt)


def to_host(t) -> np.ndarray:
    torch = torch_mod()
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy().astype(np.complex128)


def rel_l2(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def centred_shift(band, dmmap, L, dt, halo):
    """Window shift at the middle of the band's group-delay range over L and
    over the map's spans (the oracle's range), clamped to +-halo/2."""
    import oracle as O
    r = [O.group_delay_range(band, b2, b3) for b2, b3 in zip(dmmap.beta2, dmmap.beta3)]
    c = round(0.5 * (min(x[0] for x in r) + max(x[1] for x in r)) * L / dt)
    return int(max(-(halo // 2), min(halo // 2, c)))


def say(*args):
    """Name the case before a GPU step (flushed, so a fault still shows it)."""
    print("[gpu-case]", *args, file=sys.stderr, flush=True)
