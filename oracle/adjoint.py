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
* V_j is proportional to sigma_j, and the dispersion enters only through
  the phases e^{+-i theta_j}, theta_j = omega^2 B2_j / 2 + omega^3 B3_j / 6
  with B2_j = int_{z0}^{z_j} beta2 (B3_j likewise): d theta_j / d B2_j =
  omega^2 / 2.  With coefficients constant over the step B2_j = beta2 z_j
  and sigma_j = sigma.  A step across span boundaries (coefficients varying
  inside it, the generalisation before Eq. 4) has B2_j = sum_s beta2_s
  len_{j,s} (len_{j,s} the length of [z0, z_j] inside span s) and sigma_j =
  sum_s w_{j,s} sigma_s (w = 1 for the node's span, 1/2 for each side of a
  node on a boundary): its per-span derivatives are the per-node ones
  contracted with len and w.

Parity pinned by central finite differences of the forward oracle
(tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import math

import numpy as np

from .nlse import (MASK_PASS, MASK_STOP, NYQ_PASS, NYQ_STOP, _amp_every, _raised_cosine_drop,
                   block_mask, block_partition, block_taper, omega_grid, paper_fft, paper_ifft)


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


def mpa_long_step_vjp_nodes(a_z0, omega, beta2, beta3, sigma, gamma, L, M, n_iter, g_out,
                            out_mask=None, mask_grad=None, int_g=None, node_beta=None,
                            node_sigma=None):
    """Gradient of l through one long step of ``nlse.mpa_long_step``, with the
    parameter derivatives taken per node.

    The step depends on its coefficients only through the integrals
    B2_j = int_{z0}^{z_j} beta2 and B3_j (the phases theta_j = omega^2 B2_j / 2 +
    omega^3 B3_j / 6), the node values sigma_j, and, through the block roll-off,
    the step's mean coefficients B2_M / L and B3_M / L.  Returns (G(a_z0),
    dl/dsigma_j, dl/dB2_j, dl/dB3_j) for j = 0..M.  ``node_beta`` and
    ``node_sigma`` as in ``nlse.mpa_long_step`` (default: B2_j = beta2 z_j,
    B3_j = beta3 z_j, sigma_j = sigma); ``mask_grad`` = the derivatives of
    ``out_mask`` with respect to the mean coefficients (``block_mask_grad``)."""
    n = a_z0.shape[0]
    dz = L / M
    zj = dz * np.arange(M + 1)
    if node_beta is None:
        b2n, b3n = beta2 * zj, beta3 * zj
    else:
        b2n, b3n = np.asarray(node_beta[0], dtype=float), np.asarray(node_beta[1], dtype=float)
    sig = np.full(M + 1, float(sigma)) if node_sigma is None else np.asarray(node_sigma, dtype=float)
    w2, w3 = omega ** 2 / 2.0, omega ** 3 / 6.0   # d theta / d B2, d theta / d B3
    beta = np.outer(b2n, w2) + np.outer(b3n, w3)
    int_g = -gamma * zj if int_g is None else np.asarray(int_g, dtype=float)
    to_a = np.exp(1j * beta + int_g[:, None])
    to_psi = np.exp(-1j * beta - int_g[:, None])
    mask = np.ones(n) if out_mask is None else out_mask

    # forward, keeping every sweep's node spectra, time fields and V / sigma_j
    psi0 = paper_fft(a_z0)
    psis, times, vus = [], [], []
    psi = np.repeat(psi0[None, :], M + 1, axis=0)
    for _ in range(n_iter):
        psis.append(psi)
        a_t = paper_ifft(psi * to_a, axis=1)
        vu = paper_fft(np.abs(a_t) ** 2 * a_t, axis=1) * dz * to_psi
        v = sig[:, None] * vu
        times.append(a_t)
        vus.append(vu)
        csum = np.cumsum(v, axis=0)
        new = np.empty_like(psi)
        new[0] = psi0
        new[1:] = psi0[None, :] + 1j * (csum[1:] - 0.5 * v[0][None, :] - 0.5 * v[1:])
        psi = new
    x_out = psi[M] * to_a[M] * mask

    d_sig = np.zeros(M + 1)
    d_b2 = np.zeros(M + 1)
    d_b3 = np.zeros(M + 1)
    # reconstruction (step 7): out = F^{-1}[x_out]
    g_x = paper_fft(g_out) / n
    d_b2[M] += float(np.real(np.sum(np.conj(g_x) * 1j * w2 * x_out)))
    d_b3[M] += float(np.real(np.sum(np.conj(g_x) * 1j * w3 * x_out)))
    if mask_grad is not None:
        x_unmasked = psi[M] * to_a[M]
        d_b2[M] += float(np.real(np.sum(np.conj(g_x) * mask_grad[0] * x_unmasked))) / L
        d_b3[M] += float(np.real(np.sum(np.conj(g_x) * mask_grad[1] * x_unmasked))) / L
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
        # V_j = sigma_j dz to_psi_j F[|A|^2 A], A = F^{-1}[psi^(s)_j to_a_j]
        vu, a_t, ps = vus[s], times[s], psis[s]
        v = sig[:, None] * vu
        d_sig += np.real(np.sum(np.conj(g_v) * vu, axis=1))
        d_b2 += np.real(np.sum(np.conj(g_v) * (-1j) * w2 * v, axis=1))
        d_b3 += np.real(np.sum(np.conj(g_v) * (-1j) * w3 * v, axis=1))
        g_y = np.conj(sig[:, None] * dz * to_psi) * g_v
        g_n = n * paper_ifft(g_y, axis=1)
        g_a = 2 * np.abs(a_t) ** 2 * g_n + a_t ** 2 * np.conj(g_n)
        g_xn = paper_fft(g_a, axis=1) / n
        x = ps * to_a
        d_b2 += np.real(np.sum(np.conj(g_xn) * 1j * w2 * x, axis=1))
        d_b3 += np.real(np.sum(np.conj(g_xn) * 1j * w3 * x, axis=1))
        g_prev = np.conj(to_a) * g_xn
        if s == 0:
            g_psi0 += g_prev.sum(axis=0)
        else:
            g_psi = g_prev
    g_a0 = n * paper_ifft(g_psi0)
    return g_a0, d_sig, d_b2, d_b3


def mpa_long_step_vjp(a_z0, omega, beta2, beta3, sigma, gamma, L, M, n_iter, g_out,
                      out_mask=None, mask_grad=None, int_g=None):
    """Gradient of l through one long step of ``nlse.mpa_long_step`` with
    coefficients constant over the step.

    Returns (G(a_z0), dl/dsigma, dl/dbeta2, dl/dbeta3) given G(out) = g_out:
    the per-node derivatives of ``mpa_long_step_vjp_nodes`` contracted with
    dB2_j / dbeta2 = z_j (the same for beta3) and dsigma_j / dsigma = 1.
    ``mask_grad`` = (d out_mask / d beta2, d out_mask / d beta3) when the
    output mask depends on the dispersion."""
    g_a0, d_sig, d_b2, d_b3 = mpa_long_step_vjp_nodes(
        a_z0, omega, beta2, beta3, sigma, gamma, L, M, n_iter, g_out, out_mask=out_mask,
        mask_grad=mask_grad, int_g=int_g)
    zj = (L / M) * np.arange(M + 1)
    return g_a0, float(np.sum(d_sig)), float(np.dot(zj, d_b2)), float(np.dot(zj, d_b3))


def mpa_blocked_long_step_vjp(a_z0, dt, block, halo, beta2, beta3, sigma, gamma, L, M,
                              n_iter, g_out, int_g=None, shift=0, node_beta=None, node_sigma=None):
    """VJP of ``nlse.mpa_blocked_long_step`` (tapered windows, roll-off,
    cores stitched): window gradients are the core of g_out, zero elsewhere;
    the input gradient adds every window's contribution.  Returns (G(a_z0),
    dl/dsigma_j, dl/dB2_j, dl/dB3_j), the parameter derivatives per node as in
    ``mpa_long_step_vjp_nodes``."""
    n = a_z0.shape[0]
    if block == 0 or (block == n and halo == 0):
        return mpa_long_step_vjp_nodes(a_z0, omega_grid(n, dt), beta2, beta3, sigma, gamma, L, M,
                                       n_iter, g_out, int_g=int_g, node_beta=node_beta,
                                       node_sigma=node_sigma)
    omega_b = omega_grid(block, dt)
    taper = block_taper(block, halo)
    bet2, bet3 = beta2, beta3
    if node_beta is not None:      # the roll-off follows the step's mean coefficients
        bet2, bet3 = node_beta[0][-1] / L, node_beta[1][-1] / L
    mask = block_mask(omega_b, bet2, bet3, L, halo, dt, shift) if halo > 0 else None
    mask_grad = block_mask_grad(omega_b, bet2, bet3, L, halo, dt, shift) if halo > 0 else None
    g_in = np.zeros(n, dtype=np.complex128)
    ds = np.zeros(M + 1)
    d2 = np.zeros(M + 1)
    d3 = np.zeros(M + 1)
    lead = halo + shift
    for w0, c0, clen in block_partition(n, block, halo, shift):
        idx = (w0 + np.arange(block)) % n
        gw = np.zeros(block, dtype=np.complex128)
        gw[lead:lead + clen] = g_out[c0:c0 + clen]
        ga, s_, b2_, b3_ = mpa_long_step_vjp_nodes(
            a_z0[idx] * taper, omega_b, beta2, beta3, sigma, gamma, L, M, n_iter, gw,
            out_mask=mask, mask_grad=mask_grad, int_g=int_g, node_beta=node_beta,
            node_sigma=node_sigma)
        np.add.at(g_in, idx, taper * ga)
        ds += s_
        d2 += b2_
        d3 += b3_
    return g_in, ds, d2, d3


def step_weights(dmmap, L: float, M: int, m: int):
    """For long step m and every span s: len[s, j], the length of [z0, z_j]
    inside span s (d B2_j / d beta2_s), and w[s, j], the weight of sigma_s in
    sigma_j (d sigma_j / d sigma_s) -- the derivatives of
    ``nlse.step_coefficients``, which equal sum_s beta2_s len[s] and
    sum_s sigma_s w[s].  A step inside one span s (``nlse.mpa_step`` runs it
    with that span's constant coefficients, also on a node that lies on the
    span's ends) has len[s] = z_j - z0 = j dz and w[s] = 1."""
    from .nlse import long_step_spans
    nseg = len(dmmap.seg_len)
    spans = long_step_spans(dmmap, L, m)
    if len(spans) == 1:
        lens = np.zeros((nseg, M + 1))
        ws = np.zeros((nseg, M + 1))
        lens[spans[0]] = (L / M) * np.arange(M + 1)
        ws[spans[0]] = 1.0
        return lens, ws
    period = float(sum(dmmap.seg_len))
    steps = int(round(period / L))
    z0 = (m % steps) * L
    zj = z0 + (L / M) * np.arange(M + 1)
    bounds = np.concatenate([[0.0], np.cumsum(dmmap.seg_len)])
    lens = np.zeros((nseg, M + 1))
    ws = np.zeros((nseg, M + 1))
    for i in range(nseg):
        lo, hi = bounds[i], bounds[i + 1]
        lens[i] = np.clip(zj, lo, hi) - np.clip(z0, lo, hi)
    eps = 1e-12 * period
    for j, z in enumerate(zj):
        k = int(np.argmin(np.abs(bounds - z)))
        if abs(bounds[k] - z) <= eps:                          # on a boundary (periodic map)
            ws[(k - 1) % nseg, j] += 0.5
            ws[k % nseg, j] += 0.5
        else:
            ws[int(np.searchsorted(bounds, z, side="right")) - 1, j] = 1.0
    return lens, ws


def mpa_propagate_vjp(a, dt, dmmap, L, M, n_iter, z0, z1, g_out, block=0, halo=0, shift=0):
    """Gradient through ``nlse.mpa_propagate``: returns (G(a), dl/dsigma per
    span, dl/dbeta2 per span, dl/dbeta3 per span).  The forward is re-run
    storing the input of every long step; each step's per-node derivatives
    are contracted with ``step_weights``."""
    from .nlse import (_grid_index, long_step_gain, long_step_spans, lumped_gain, mpa_step,
                       step_coefficients)
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
        if every and (m + 1) % every == 0:
            g = g * lumped_gain(dmmap)
        spans = long_step_spans(dmmap, L, m)
        int_g = long_step_gain(dmmap, L, M, m)
        if len(spans) == 1:
            s = spans[0]
            g, ds, d2, d3 = mpa_blocked_long_step_vjp(
                inputs[m - m0], dt, block or len(a), halo, dmmap.beta2[s], dmmap.beta3[s],
                dmmap.sigma[s], dmmap.gamma, L, M, n_iter, g, int_g=int_g, shift=shift)
        else:
            node_beta, node_sigma = step_coefficients(dmmap, L, M, m)
            g, ds, d2, d3 = mpa_blocked_long_step_vjp(
                inputs[m - m0], dt, block or len(a), halo, 0.0, 0.0, 0.0, dmmap.gamma, L, M,
                n_iter, g, int_g=int_g, shift=shift, node_beta=node_beta, node_sigma=node_sigma)
        lens, ws = step_weights(dmmap, L, M, m)
        g_sigma += ws @ ds
        g_beta2 += lens @ d2
        g_beta3 += lens @ d3
    return g, g_sigma, g_beta2, g_beta3
