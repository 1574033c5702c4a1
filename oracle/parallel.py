"""The paper's own parallel decomposition of one MPA long step, on host cores.

TEST INFRASTRUCTURE ONLY (see the package docstring): the all-core CPU
baseline of the benchmark and its pin.  Plain NumPy in complex128.

The paper distributes a long step over processors by z-node: the FFTs of
steps 3 and 4 of every node are independent within a sweep and dominate the
work, while steps 2 and 5 act harmonic by harmonic (the description of the
parallel implementation after Fig. 1).  This module runs exactly the
Jacobi sweeps of ``nlse.mpa_long_step`` (Eq. 6, steps 1-7), with

* the node evaluations of a sweep (phase, inverse transform, |A|^2 A,
  transform, conjugate phase: steps 2-4) mapped over a pool of threads, one
  node per task, and
* the cumulative trapezoid of step 5 split into contiguous ranges of
  harmonics, one range per task;

NumPy's FFT releases the interpreter lock, so the threads run on separate
cores.  Node 0 of a sweep is evaluated like every other node, as in the
paper's Jacobi form.  The arithmetic per harmonic and per node is that of
``nlse.mpa_long_step`` in the same order, so the two agree to rounding.
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

from .nlse import paper_fft, paper_ifft


def mpa_long_step_parallel(a_z0, omega, beta2, beta3, sigma, gamma, L, M, n_iter, workers=None,
                           pool=None):
    """One long step of the full-window MPA (Eq. 6) with the node work of
    each sweep and the per-harmonic trapezoid spread over ``workers``
    threads (default: every host core)."""
    workers = workers or os.cpu_count() or 1
    own = pool is None
    if own:
        pool = cf.ThreadPoolExecutor(max_workers=workers)
    try:
        n = a_z0.shape[0]
        dz = L / M
        zj = dz * np.arange(M + 1)

        def phases(j):
            beta = zj[j] * (omega ** 2 / 2.0 * beta2 + omega ** 3 / 6.0 * beta3)
            return np.exp(1j * beta - gamma * zj[j]), np.exp(-1j * beta + gamma * zj[j])

        to = list(pool.map(phases, range(M + 1)))
        psi0 = paper_fft(a_z0)                                     # step 1
        psi = [psi0] * (M + 1)
        v = [None] * (M + 1)

        def node(j):                                               # steps 2-4 at node j
            a_t = paper_ifft(psi[j] * to[j][0])
            return sigma * paper_fft(np.abs(a_t) ** 2 * a_t) * dz * to[j][1]

        cuts = np.linspace(0, n, workers + 1).astype(int)
        for _ in range(n_iter):
            v = list(pool.map(node, range(M + 1)))
            new = [None] + [np.empty(n, dtype=np.complex128) for _ in range(M)]

            def trapezoid(r):                                      # step 5 on harmonics [lo, hi)
                lo, hi = cuts[r], cuts[r + 1]
                vs = np.stack([x[lo:hi] for x in v])
                csum = np.cumsum(vs, axis=0)
                out = psi0[None, lo:hi] + 1j * (csum[1:] - 0.5 * vs[0][None, :] - 0.5 * vs[1:])
                for l in range(1, M + 1):
                    new[l][lo:hi] = out[l - 1]

            list(pool.map(trapezoid, range(workers)))
            new[0] = psi0
            psi = new                                              # step 6: next sweep
        return paper_ifft(psi[M] * to[M][0])                       # step 7
    finally:
        if own:
            pool.shutdown()
