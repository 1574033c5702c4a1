"""FP64 oracle of the gradient of the MPA (vector-Jacobian products).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Gradients of a real loss l with respect to a complex array z are packed as
G(z) = dl/dRe z + i dl/dIm z (so dl = Re sum conj(G) dz).  The adjoint
rules used, derived from the forward steps of ``nlse.mpa_long_step``
(MPA steps 1-7, Eq. 6):

* y = c z (c fixed complex): G(z) = conj(c) G(y);
* the paper's transform F (unnormalised, kernel e^{+i omega t}) has adjoint
  N F^{-1}; its inverse F^{-1} has adjoint F / N;
* n = |a|^2 a: G(a) = 2 |a|^2 G(n) + a^2 conj(G(n));
* the cumulative trapezoid psi_l = psi_0 + i (V_0/2 + sum_{0<j<l} V_j + V_l/2)
  has adjoint G(V_j) = -i (G(psi_j)/2 + sum_{l>j} G(psi_l)) (j >= 1),
  G(V_0) = -i sum_l G(psi_l) / 2 -- a reverse cumulative sum;
* V_j is proportional to sigma, and beta2 (beta3) enter only through the
  phases e^{+-i theta_j}, d theta_j / d beta2 = omega^2 z_j / 2
  (d theta_j / d beta3 = omega^3 z_j / 6).

Parity pinned by central finite differences of the forward oracle
(tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import math

import numpy as np

from .nlse import (MASK_PASS, MASK_STOP, NYQ_PASS, NYQ_STOP, _amp_every, _raised_cosine_drop,
                   block_mask, block_partition, block_taper, omega_grid, paper_fft, paper_ifft,
                   span_of_long_step)


def _raised_cosine_slope(x):
    """d/dx of ``nlse._raised_cosine_drop``: -pi/2 sin(pi x) on (0, 1), else 0."""
    return np.where((x > 0) & (x < 1), -0.5 * math.pi * np.sin(math.pi * np.clip(x, 0, 1)), 0.0)


def block_mask_grad(omega_b, beta2, beta3, L, halo, dt, shift=0):
    """Derivatives of ``nlse.block_mask`` with respect to beta2 and beta3.

    Only the first roll-off depends on them, through
    g = |u| / (halo dt), u = (beta2 omega + beta3 omega^2 / 2) L - shift dt:
    dg/dbeta2 = sign(u) omega L / (halo dt), dg/dbeta3 = sign(u) omega^2 L / (2 halo dt)."""
    u = (beta2 * omega_b + 0.5 * beta3 * omega_b ** 2) * L - shift * dt
    scale = L / (halo * dt)
    width = MASK_STOP - MASK_PASS
    x1 = (np.abs(u) / (halo * dt) - MASK_PASS) / width
    r = np.abs(omega_b) * dt / math.pi
    other = _raised_cosine_drop((r - NYQ_PASS) / (NYQ_STOP - NYQ_PASS))
    dm_dg = _raised_cosine_slope(x1) / width * other
    return dm_dg * np.sign(u) * omega_b * scale, dm_dg * np.sign(u) * 0.5 * omega_b ** 2 * scale


def mpa_long_step_vjp(a_z0, omega, beta2, beta3, sigma, gamma, L, M, n_iter, g_out,
                      out_mask=None, mask_grad=None, int_g=None):
    """Gradient of l through one long step of ``nlse.mpa_long_step``.

    Returns (G(a_z0), dl/dsigma, dl/dbeta2, dl/dbeta3) given G(out) = g_out.
    ``mask_grad`` = (d out_mask / d beta2, d out_mask / d beta3) when the
    output mask depends on the dispersion."""
    n = a_z0.shape[0]
    dz = L / M
    zj = dz * np.arange(M + 1)
    beta = np.outer(zj, omega ** 2 / 2.0 * beta2 + omega ** 3 / 6.0 * beta3)
    int_g = -gamma * zj if int_g is None else np.asarray(int_g, dtype=float)
    to_a = np.exp(1j * beta + int_g[:, None])
    to_psi = np.exp(-1j * beta - int_g[:, None])
    k2 = np.outer(zj, omega ** 2 / 2.0)          # d theta_j / d beta2
    k3 = np.outer(zj, omega ** 3 / 6.0)          # d theta_j / d beta3
    mask = np.ones(n) if out_mask is None else out_mask

    # forward, keeping every sweep's node spectra, time fields and V
    psi0 = paper_fft(a_z0)
    psis, times, vs = [], [], []
    psi = np.repeat(psi0[None, :], M + 1, axis=0)
    for _ in range(n_iter):
        psis.append(psi)
        a_t = paper_ifft(psi * to_a, axis=1)
        v = sigma * paper_fft(np.abs(a_t) ** 2 * a_t, axis=1) * dz * to_psi
        times.append(a_t)
        vs.append(v)
        csum = np.cumsum(v, axis=0)
        new = np.empty_like(psi)
        new[0] = psi0
        new[1:] = psi0[None, :] + 1j * (csum[1:] - 0.5 * v[0][None, :] - 0.5 * v[1:])
        psi = new
    x_out = psi[M] * to_a[M] * mask

    d_sigma = d_b2 = d_b3 = 0.0
    # reconstruction (step 7): out = F^{-1}[x_out]
    g_x = paper_fft(g_out) / n
    d_b2 += float(np.real(np.sum(np.conj(g_x) * 1j * k2[M] * x_out)))
    d_b3 += float(np.real(np.sum(np.conj(g_x) * 1j * k3[M] * x_out)))
    if mask_grad is not None:
        x_unmasked = psi[M] * to_a[M]
        d_b2 += float(np.real(np.sum(np.conj(g_x) * mask_grad[0] * x_unmasked)))
        d_b3 += float(np.real(np.sum(np.conj(g_x) * mask_grad[1] * x_unmasked)))
    g_psi = np.zeros((M + 1, n), dtype=np.complex128)
    g_psi[M] = np.conj(to_a[M] * mask) * g_x
    g_psi0 = np.zeros(n, dtype=np.complex128)
    for s in range(n_iter - 1, -1, -1):
        # level s+1 -> V^(s): psi^(s+1)_0 is psi_0 itself
        g_psi0 += g_psi[0]
        gl = g_psi[1:]                                   # l = 1..M
        g_psi0 += gl.sum(axis=0)
        rev = np.cumsum(gl[::-1], axis=0)[::-1]          # sum_{l >= j}
        g_v = np.empty((M + 1, n), dtype=np.complex128)
        g_v[0] = -0.5j * gl.sum(axis=0)
        g_v[1:] = -1j * (rev - 0.5 * gl)                 # G(psi_j)/2 + sum_{l>j} G(psi_l)
        # V_j = sigma dz to_psi_j F[|A|^2 A], A = F^{-1}[psi^(s)_j to_a_j]
        v, a_t, ps = vs[s], times[s], psis[s]
        d_sigma += float(np.real(np.sum(np.conj(g_v) * v))) / sigma
        d_b2 += float(np.real(np.sum(np.conj(g_v) * (-1j) * k2 * v)))
        d_b3 += float(np.real(np.sum(np.conj(g_v) * (-1j) * k3 * v)))
        g_y = np.conj(sigma * dz * to_psi) * g_v
        g_n = n * paper_ifft(g_y, axis=1)
        g_a = 2 * np.abs(a_t) ** 2 * g_n + a_t ** 2 * np.conj(g_n)
        g_xn = paper_fft(g_a, axis=1) / n
        x = ps * to_a
        d_b2 += float(np.real(np.sum(np.conj(g_xn) * 1j * k2 * x)))
        d_b3 += float(np.real(np.sum(np.conj(g_xn) * 1j * k3 * x)))
        g_prev = np.conj(to_a) * g_xn
        if s == 0:
            g_psi0 += g_prev.sum(axis=0)
        else:
            g_psi = g_prev
    g_a0 = n * paper_ifft(g_psi0)
    return g_a0, d_sigma, d_b2, d_b3


def mpa_blocked_long_step_vjp(a_z0, dt, block, halo, beta2, beta3, sigma, gamma, L, M,
                              n_iter, g_out, int_g=None, shift=0):
    """VJP of ``nlse.mpa_blocked_long_step`` (tapered windows, roll-off,
    cores stitched): window gradients are the core of g_out, zero elsewhere;
    the input gradient adds every window's contribution."""
    n = a_z0.shape[0]
    if block == 0 or (block == n and halo == 0):
        return mpa_long_step_vjp(a_z0, omega_grid(n, dt), beta2, beta3, sigma, gamma, L, M,
                                 n_iter, g_out, int_g=int_g)
    omega_b = omega_grid(block, dt)
    taper = block_taper(block, halo)
    mask = block_mask(omega_b, beta2, beta3, L, halo, dt, shift) if halo > 0 else None
    mask_grad = block_mask_grad(omega_b, beta2, beta3, L, halo, dt, shift) if halo > 0 else None
    g_in = np.zeros(n, dtype=np.complex128)
    ds = d2 = d3 = 0.0
    lead = halo + shift
    for w0, c0, clen in block_partition(n, block, halo, shift):
        idx = (w0 + np.arange(block)) % n
        gw = np.zeros(block, dtype=np.complex128)
        gw[lead:lead + clen] = g_out[c0:c0 + clen]
        ga, s_, b2_, b3_ = mpa_long_step_vjp(a_z0[idx] * taper, omega_b, beta2, beta3, sigma,
                                             gamma, L, M, n_iter, gw, out_mask=mask,
                                             mask_grad=mask_grad, int_g=int_g)
        np.add.at(g_in, idx, taper * ga)
        ds += s_
        d2 += b2_
        d3 += b3_
    return g_in, ds, d2, d3


def mpa_propagate_vjp(a, dt, dmmap, L, M, n_iter, z0, z1, g_out, block=0, halo=0, shift=0):
    """Gradient through ``nlse.mpa_propagate``: returns (G(a), dl/dsigma per
    span, dl/dbeta2 per span, dl/dbeta3 per span).  The forward is re-run storing the input of
    every long step."""
    from .nlse import _grid_index, long_step_gain, lumped_gain, mpa_step
    m0, m1 = _grid_index(z0, L), _grid_index(z1, L)
    inputs = []
    for m in range(m0, m1):
        inputs.append(a)
        a = mpa_step(a, dt, dmmap, L, M, n_iter, m, block, halo, shift)
    nspan = len(dmmap.seg_len)
    g_sigma = np.zeros(nspan)
    g_beta2 = np.zeros(nspan)
    g_beta3 = np.zeros(nspan)
    every = _amp_every(dmmap, L)
    g = g_out
    for m in range(m1 - 1, m0 - 1, -1):
        s = span_of_long_step(dmmap, L, m)
        if every and (m + 1) % every == 0:
            g = g * lumped_gain(dmmap)
        g, ds, d2, d3 = mpa_blocked_long_step_vjp(
            inputs[m - m0], dt, block or len(a), halo, dmmap.beta2[s], dmmap.beta3[s],
            dmmap.sigma[s], dmmap.gamma, L, M, n_iter, g, int_g=long_step_gain(dmmap, L, M, m),
            shift=shift)
        g_sigma[s] += ds
        g_beta2[s] += d2
        g_beta3[s] += d3
    return g, g_sigma, g_beta2, g_beta3
