"""FP64 oracle: MPA (full window and time-blocked), split-step, references.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy in
complex128; slow on purpose; each function cites the passage it follows.

Model (Eq. 1): i A_z - (1/2) beta2 A_tt - (i/6) beta3 A_ttt + sigma |A|^2 A
= i G A with G = -gamma between lumped amplifiers spaced z_a apart.

Readings taken where the paper is silent or garbled:

* Fourier pair: the paper's transform has kernel e^{+i omega t} (definition
  after Eq. 1).  On the grid t_n = n dt, omega_k = 2 pi fftfreq(N, dt)_k it is
  F[A]_k = sum_n A_n e^{+i omega_k t_n} = N * ifft(A), with inverse
  fft(.)/N.  With this pair beta(omega, z) is used exactly as printed.
* The Nyquist harmonic takes omega = -pi/dt (fftfreq's choice).
* The lumped gain factor exp(gamma z_a) is a multiplicative jump applied
  after the long step (or split-step run) that ends on an amplifier; the
  delta-function form read literally would not restore the span loss.
* beta and the integral of G are measured from the current long step's z0
  (the paper restarts with z0 = (m+1) L); all coefficients are those of the
  span that contains the long step (long steps never straddle spans).
* Span and amplifier membership are decided with integer step counters.
* n_iter counts Picard sweeps: psi^(n_iter) needs n_iter evaluations of V.
"""
from __future__ import annotations

import collections
import math
from typing import List, Sequence, Tuple

import numpy as np

DMMapSpec = collections.namedtuple(
    "DMMapSpec", "seg_len beta2 beta3 sigma gamma z_amp")


# --------------------------------------------------------------------------
# Fourier transform and frequency grid (definition after Eq. 1)
# --------------------------------------------------------------------------

def paper_fft(a: np.ndarray, axis: int = -1) -> np.ndarray:
    """F[A]_k = sum_n A_n exp(+i omega_k t_n) (the paper's transform)."""
    n = a.shape[axis]
    return n * np.fft.ifft(a, axis=axis)


def paper_ifft(ahat: np.ndarray, axis: int = -1) -> np.ndarray:
    """Inverse of :func:`paper_fft`: A_n = (1/N) sum_k Ahat_k exp(-i omega_k t_n)."""
    n = ahat.shape[axis]
    return np.fft.fft(ahat, axis=axis) / n


def omega_grid(n: int, dt: float) -> np.ndarray:
    """omega_k = 2 pi k'/(N dt) with k' the signed harmonic index."""
    return 2.0 * math.pi * np.fft.fftfreq(n, dt)


def beta_phase(omega: np.ndarray, beta2: float, beta3: float, z: float) -> np.ndarray:
    """beta(omega, z) of Eq. 2 for coefficients constant over [z0, z0 + z]."""
    return (omega ** 2 / 2.0 * beta2 + omega ** 3 / 6.0 * beta3) * z


def linear_step(a: np.ndarray, omega: np.ndarray, beta2: float, beta3: float,
                gamma: float, h: float) -> np.ndarray:
    """Exact linear propagation over h (sigma = 0 in Eq. 1): the spectrum is
    multiplied by exp(i beta(omega, h) + int G) with int G = -gamma h."""
    return paper_ifft(paper_fft(a) * np.exp(1j * beta_phase(omega, beta2, beta3, h) - gamma * h))


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


# --------------------------------------------------------------------------
# One long step of the MPA on one periodic window (Eq. 6, steps 1-7)
# --------------------------------------------------------------------------

def mpa_long_step(a_z0: np.ndarray, omega: np.ndarray, beta2: float, beta3: float,
                  sigma: float, gamma: float, L: float, M: int, n_iter: int,
                  return_iterates: bool = False, out_mask=None, int_g=None,
                  node_beta=None, node_sigma=None):
    """Advance A(t, z0) to A(t, z0 + L) by n_iter Picard sweeps of the
    discretised integral equation, Eq. 6, in the order of MPA steps 1-7.

    Nodes z_j = z0 + j dz, dz = L/M, j = 0..M.  The Jacobi form of the paper
    is kept: every sweep evaluates all nodes from the previous sweep's
    psi^(n)_j, then the trapezoid sums are formed for every l.  ``int_g``
    (M + 1 values of int_{z0}^{z_j} G) replaces -gamma (z_j - z0) when G
    is not constant (distributed gain, :func:`gain_integral`).  When the
    long step crosses a span boundary, ``node_beta`` = (int_{z0}^{z_j} beta2,
    int_{z0}^{z_j} beta3) for j = 0..M replaces (beta2, beta3) (z_j - z0)
    in beta(omega, z_j), and ``node_sigma`` (M + 1 values) replaces sigma at
    the nodes (:func:`step_coefficients`).
    """
    dz = L / M
    zj = dz * np.arange(M + 1)                                    # z_j - z0
    if node_beta is None:
        beta = np.outer(zj, omega ** 2 / 2.0 * beta2 + omega ** 3 / 6.0 * beta3)
    else:
        beta = (np.outer(node_beta[0], omega ** 2 / 2.0) + np.outer(node_beta[1], omega ** 3 / 6.0))
    sig = sigma if node_sigma is None else np.asarray(node_sigma, dtype=float)[:, None]
    int_g = -gamma * zj if int_g is None else np.asarray(int_g, dtype=float)   # int_{z0}^{z_j} G
    to_a = np.exp(1j * beta + int_g[:, None])                     # e^{+i beta + int G}
    to_psi = np.exp(-1j * beta - int_g[:, None])                  # e^{-i beta - int G}

    # step 1: psi(omega, z0) = Ahat(omega, z0), copied to every node
    psi0 = paper_fft(a_z0)
    psi = np.repeat(psi0[None, :], M + 1, axis=0)
    iterates = [psi[M].copy()]
    for _ in range(n_iter):
        a_hat = psi * to_a                                        # step 2
        a_t = paper_ifft(a_hat, axis=1)                           # step 3
        v = sig * paper_fft(np.abs(a_t) ** 2 * a_t, axis=1) * dz * to_psi     # step 4, V_j of Eq. 6
        # step 5: trapezoid rule, Eq. 6, saving the partial integral at every node:
        # psi_l = psi_0 + i (V_0/2 + sum_{j=1}^{l-1} V_j + V_l/2), l = 1..M
        csum = np.cumsum(v, axis=0)                               # sum_{j=0}^{l} V_j
        new = np.empty_like(psi)
        new[0] = psi0
        new[1:] = psi0[None, :] + 1j * (csum[1:] - 0.5 * v[0][None, :] - 0.5 * v[1:])
        psi = new                                                 # step 6: next sweep
        iterates.append(psi[M].copy())
    spec = psi[M] * to_a[M]                                      # step 7
    if out_mask is not None:
        spec = spec * out_mask
    out = paper_ifft(spec)
    if return_iterates:
        return out, iterates
    return out


def if_trapezoid_long_step(a_z0: np.ndarray, omega: np.ndarray, beta2: float,
                           beta3: float, sigma: float, gamma: float, L: float,
                           M: int, tol: float = 1e-15, max_iter: int = 500) -> np.ndarray:
    """The sequential implicit trapezoid rule for the integral equation
    (Eq. 2) in the interaction picture:
        psi_l = psi_{l-1} + (i dz / 2) (f(z_{l-1}, psi_{l-1}) + f(z_l, psi_l)),
    f(z, psi) = sigma e^{-i beta - int G} F[|A|^2 A], A = F^{-1}[psi e^{i beta + int G}],
    each node solved by fixed-point iteration.  This is the n -> infinity
    limit that Eq. 6 approaches (a check of the MPA's summation)."""
    dz = L / M

    def f(z, psi):
        ph = 1j * beta_phase(omega, beta2, beta3, z) - gamma * z
        a = paper_ifft(psi * np.exp(ph))
        return sigma * paper_fft(np.abs(a) ** 2 * a) * np.exp(-ph)

    psi = paper_fft(a_z0)
    f_prev = f(0.0, psi)
    for l in range(1, M + 1):
        z = l * dz
        x = psi.copy()
        for _ in range(max_iter):
            fx = f(z, x)
            x_new = psi + 0.5j * dz * (f_prev + fx)
            done = np.max(np.abs(x_new - x)) <= tol * np.max(np.abs(x_new))
            x = x_new
            if done:
                break
        psi = x
        f_prev = f(z, psi)
    ph = 1j * beta_phase(omega, beta2, beta3, L) - gamma * L
    return paper_ifft(psi * np.exp(ph))


# --------------------------------------------------------------------------
# Time blocking (not in the paper; the partition rule the library uses)
# --------------------------------------------------------------------------

def block_partition(n: int, block: int, halo: int, shift: int = 0) -> List[Tuple[int, int, int]]:
    """Blocks of ``block`` samples overlapping by ``2 halo``.

    Block b owns the core [b C, min((b+1) C, n)) with C = block - 2 halo and
    reads the periodic window starting at b C - halo - shift: the core sits
    halo + shift samples into its window, so a window shift moves the window
    towards earlier times by ``shift`` samples (halo + shift before the core,
    halo - shift after it).  Content travels towards later times when its
    group delay beta2 omega + beta3 omega^2 / 2 is positive, so a shift near
    the middle of the band's group delay over L keeps the core's domain of
    dependence centred in its window.  Returns (window_start, core_start,
    core_len) per block.  block = n (halo = 0) gives the single full window.
    """
    if block == n and halo == 0:
        return [(0, 0, n)]
    core = block - 2 * halo
    nb = -(-n // core)
    out = []
    for b in range(nb):
        c0 = b * core
        out.append((c0 - halo - shift, c0, min(core, n - c0)))
    return out


TAPER_STEEPNESS = 8.0


def block_taper(block: int, halo: int) -> np.ndarray:
    """Weights applied to a block window before its first transform.

    A window cut out of the field is not periodic: the jump where its two
    ends meet carries content up to the grid's Nyquist frequency, which
    dispersion carries across any practical halo within one long step.  The
    outer W = halo // 2 samples of each side are therefore rolled off with
    s(x) = (1 + erf(8 (x - 1/2))) / 2, x = (i + 1/2) / W (i counted from the
    window edge); the rest of the window, and so the core and the inner half
    of each halo, is untouched.  halo = 0 gives all ones."""
    w = np.ones(block)
    W = halo // 2
    if W > 0:
        x = (np.arange(W) + 0.5) / W
        s = np.array([0.5 * (1.0 + math.erf(TAPER_STEEPNESS * (xi - 0.5))) for xi in x])
        w[:W] = s
        w[block - W:] = s[::-1]
    return w


MASK_PASS = 0.35       # group delay over L, in units of the halo duration
MASK_STOP = 0.5
NYQ_PASS = 0.8         # |omega| in units of the grid's Nyquist frequency pi/dt
NYQ_STOP = 0.9


def _raised_cosine_drop(x: np.ndarray) -> np.ndarray:
    """1 for x <= 0, 0 for x >= 1, (1 + cos(pi x)) / 2 in between."""
    return np.where(x <= 0, 1.0, np.where(x >= 1, 0.0, 0.5 * (1.0 + np.cos(math.pi * np.clip(x, 0, 1)))))


def block_mask(omega_b: np.ndarray, beta2: float, beta3: float, L: float, halo: int,
               dt: float, shift: int = 0) -> np.ndarray:
    """Spectral roll-off applied to each block's spectrum when it is
    reconstructed (step 7 of a blocked long step).

    Stitching overlapping periodic windows is not a unitary map, and two
    kinds of content grow under it by a fixed factor every long step even
    with sigma = 0: content whose group delay over L carries it into the
    tapered outer halo, and, when beta3 != 0, content at the grid's Nyquist
    frequency, where the odd beta3 term makes beta(omega) jump between
    +pi/dt and -pi/dt.  The mask is the product of two raised-cosine
    roll-offs: in g = |(beta2 omega + beta3 omega^2 / 2) L - shift dt| / (halo dt)
    (the displacement of content over the long step relative to the window
    shift, in units of the halo duration), from 1 at g = 0.35 to 0 at
    g = 0.5 (the halo rule keeps the signal band at g <= 0.25), and in
    |omega| dt / pi, from 1 at 0.8 to 0 at 0.9."""
    g = np.abs((beta2 * omega_b + 0.5 * beta3 * omega_b ** 2) * L - shift * dt) / (halo * dt)
    r = np.abs(omega_b) * dt / math.pi
    return (_raised_cosine_drop((g - MASK_PASS) / (MASK_STOP - MASK_PASS))
            * _raised_cosine_drop((r - NYQ_PASS) / (NYQ_STOP - NYQ_PASS)))


def mpa_blocked_long_step(a_z0: np.ndarray, dt: float, block: int, halo: int,
                          beta2: float, beta3: float, sigma: float, gamma: float,
                          L: float, M: int, n_iter: int, int_g=None, node_beta=None,
                          node_sigma=None, shift: int = 0) -> np.ndarray:
    """One MPA long step run independently on every periodic block window
    (frequency grid of the block: omega^B = 2 pi fftfreq(block, dt)), keeping
    each block's core.  Each window is multiplied by :func:`block_taper`
    first and each block's final spectrum by :func:`block_mask`.  ``shift``
    moves every window against its core (see :func:`block_partition`); the
    core must stay clear of the tapered outer halo/2 samples, |shift| <= halo/2."""
    n = a_z0.shape[0]
    if block == 0 or (block == n and halo == 0):
        return mpa_long_step(a_z0, omega_grid(n, dt), beta2, beta3, sigma, gamma,
                             L, M, n_iter, int_g=int_g, node_beta=node_beta, node_sigma=node_sigma)
    if abs(shift) > halo // 2:
        raise ValueError(f"window shift {shift} exceeds halo/2 = {halo // 2}")
    omega_b = omega_grid(block, dt)
    taper = block_taper(block, halo)
    bet2, bet3 = beta2, beta3
    if node_beta is not None:      # the step's group delay: integrated coefficients over L
        bet2, bet3 = node_beta[0][-1] / L, node_beta[1][-1] / L
    mask = block_mask(omega_b, bet2, bet3, L, halo, dt, shift) if halo > 0 else None
    out = np.empty_like(a_z0)
    lead = halo + shift
    for w0, c0, clen in block_partition(n, block, halo, shift):
        idx = (w0 + np.arange(block)) % n
        res = mpa_long_step(a_z0[idx] * taper, omega_b, beta2, beta3, sigma, gamma,
                            L, M, n_iter, out_mask=mask, int_g=int_g, node_beta=node_beta,
                            node_sigma=node_sigma)
        out[c0:c0 + clen] = res[lead:lead + clen]
    return out


def halo_rate(omega_band: float, beta2: float, beta3: float) -> float:
    """Largest group-delay rate |beta2 omega + beta3 omega^2 / 2| over
    |omega| <= omega_band (time shift per unit z of the fastest content)."""
    return abs(beta2) * omega_band + 0.5 * abs(beta3) * omega_band ** 2


def group_delay_range(omega_band: float, beta2: float, beta3: float):
    """(min, max) of the group-delay rate beta2 omega + beta3 omega^2 / 2 over
    |omega| <= omega_band: the values at both band edges and, when the
    parabola's vertex -beta2/beta3 lies inside the band, at the vertex."""
    w = float(omega_band)
    vals = [beta2 * w + 0.5 * beta3 * w * w, -beta2 * w + 0.5 * beta3 * w * w]
    if beta3 != 0 and abs(beta2 / beta3) <= w:
        vals.append(-0.5 * beta2 * beta2 / beta3)
    return min(vals), max(vals)


def halo_excursion(omega_band: float, beta2: float, beta3: float, L: float, shift: int,
                   dt: float) -> float:
    """Largest displacement over one long step of content in the band,
    relative to the window shift: max |(beta2 omega + beta3 omega^2 / 2) L -
    shift dt| over |omega| <= omega_band (its extremes lie at the ends of the
    group-delay range)."""
    lo, hi = group_delay_range(omega_band, beta2, beta3)
    return max(abs(lo * L - shift * dt), abs(hi * L - shift * dt))


# --------------------------------------------------------------------------
# Marching over the map (long steps z0 = m L, MPA steps 1-7 per interval)
# --------------------------------------------------------------------------

def _steps_per(length: float, h: float, what: str) -> int:
    k = int(round(length / h))
    if k < 1 or abs(k * h - length) > 1e-9 * max(length, h):
        raise ValueError(f"step {h} does not divide {what} {length}")
    return k


def span_of_long_step(dmmap, h: float, m: int) -> int:
    """Index of the span containing step m of length h (integer counters)."""
    counts = [_steps_per(s, h, "span") for s in dmmap.seg_len]
    r = m % sum(counts)
    for i, c in enumerate(counts):
        if r < c:
            return i
        r -= c
    raise AssertionError


def long_step_spans(dmmap, L: float, m: int):
    """Spans overlapped by long step m ([mL, (m+1)L]) when L divides the map
    period but not necessarily every span."""
    period = float(sum(dmmap.seg_len))
    steps = _steps_per(period, L, "map period")
    z0 = (m % steps) * L
    bounds = np.concatenate([[0.0], np.cumsum(dmmap.seg_len)])
    eps = 1e-12 * period
    return [i for i in range(len(dmmap.seg_len))
            if bounds[i] < z0 + L - eps and bounds[i + 1] > z0 + eps]


def step_coefficients(dmmap, L: float, M: int, m: int):
    """For long step m: int_{z0}^{z_j} beta2 and beta3 (exact integrals of the
    piecewise-constant map) and sigma at the nodes z_j, j = 0..M.  A node on a
    span boundary takes the mean of the two spans' sigma: the trapezoid rule
    then equals the trapezoid rule applied on each side of the boundary."""
    period = float(sum(dmmap.seg_len))
    steps = _steps_per(period, L, "map period")
    z0 = (m % steps) * L
    zj = z0 + (L / M) * np.arange(M + 1)
    bounds = np.concatenate([[0.0], np.cumsum(dmmap.seg_len)])
    b2 = np.zeros(M + 1)
    b3 = np.zeros(M + 1)
    for i in range(len(dmmap.seg_len)):
        lo, hi = bounds[i], bounds[i + 1]
        seg = np.clip(zj, lo, hi) - np.clip(z0, lo, hi)         # length of [z0, z_j] inside span i
        b2 += dmmap.beta2[i] * seg
        b3 += dmmap.beta3[i] * seg
    eps = 1e-12 * period
    nseg = len(dmmap.seg_len)
    sig = np.empty(M + 1)
    for j, z in enumerate(zj):
        k = int(np.argmin(np.abs(bounds - z)))
        if abs(bounds[k] - z) <= eps:                          # on a boundary (periodic map)
            left, right = (k - 1) % nseg, k % nseg
            sig[j] = 0.5 * (dmmap.sigma[left] + dmmap.sigma[right])
        else:
            sig[j] = dmmap.sigma[int(np.searchsorted(bounds, z, side="right")) - 1]
    return (b2, b3), sig


def _amp_every(dmmap, h: float) -> int:
    if dmmap.z_amp <= 0:
        return 0
    return _steps_per(dmmap.z_amp, h, "amplifier spacing")


def _raman(dmmap):
    g0 = float(getattr(dmmap, "raman_g0", 0.0) or 0.0)
    return g0, float(getattr(dmmap, "raman_alpha", 0.0) or 0.0)


def gain_integral(dmmap, zeta0: float, h) -> np.ndarray:
    """int_{z0}^{z0 + h} G(z) dz for a start z0 whose position inside its
    amplifier period is zeta0 (0 <= zeta0 < z_a), for offsets h >= 0 that stay
    inside that period.

    G(z) = -gamma + g(z) (Eq. 1 allows any G): the loss plus an optional
    distributed, backward-pumped gain rising towards each amplifier,
    g = g0 exp(-alpha (z_a - zeta)) at position zeta of the amplifier period,
    whose integral is (g0 / alpha) (exp(-alpha (z_a - zeta0 - h)) -
    exp(-alpha (z_a - zeta0)))."""
    h = np.asarray(h, dtype=float)
    out = -dmmap.gamma * h
    g0, alpha = _raman(dmmap)
    if g0 > 0:
        za = dmmap.z_amp
        out = out + (g0 / alpha) * (np.exp(-alpha * (za - zeta0 - h)) - np.exp(-alpha * (za - zeta0)))
    return out


def lumped_gain(dmmap) -> float:
    """Amplitude factor of a lumped amplifier: it makes up what the span
    loss and the distributed gain leave over one amplifier period,
    exp(gamma z_a - int_0^{z_a} g), so that the link is transparent."""
    g0, alpha = _raman(dmmap)
    dist = (g0 / alpha) * (1.0 - math.exp(-alpha * dmmap.z_amp)) if g0 > 0 else 0.0
    return math.exp(dmmap.gamma * dmmap.z_amp - dist)


def long_step_gain(dmmap, L: float, M: int, m: int):
    """int_{mL}^{mL + j dz} G for j = 0..M (None when G = -gamma throughout)."""
    g0, _ = _raman(dmmap)
    if g0 <= 0:
        return None
    every = _amp_every(dmmap, L)
    zeta0 = (m % every) * L
    return gain_integral(dmmap, zeta0, (L / M) * np.arange(M + 1))


def mpa_step(a: np.ndarray, dt: float, dmmap, L: float, M: int, n_iter: int,
             m: int, block: int = 0, halo: int = 0, shift: int = 0) -> np.ndarray:
    """Long step m ([m L, (m+1) L]), then the lumped gain if an amplifier
    sits at (m+1) L (exp(gamma z_a) without distributed gain)."""
    spans = long_step_spans(dmmap, L, m)
    if len(spans) == 1:
        s = spans[0]
        out = mpa_blocked_long_step(a, dt, block or a.shape[0], halo, dmmap.beta2[s],
                                    dmmap.beta3[s], dmmap.sigma[s], dmmap.gamma,
                                    L, M, n_iter, int_g=long_step_gain(dmmap, L, M, m), shift=shift)
    else:
        # the step crosses a span boundary: exact beta integrals, sigma sampled at the nodes
        node_beta, node_sigma = step_coefficients(dmmap, L, M, m)
        out = mpa_blocked_long_step(a, dt, block or a.shape[0], halo, 0.0, 0.0, 0.0, dmmap.gamma,
                                    L, M, n_iter, int_g=long_step_gain(dmmap, L, M, m),
                                    node_beta=node_beta, node_sigma=node_sigma, shift=shift)
    every = _amp_every(dmmap, L)
    if every and (m + 1) % every == 0:
        out = out * lumped_gain(dmmap)
    return out


def _grid_index(z: float, h: float) -> int:
    m = int(round(z / h))
    if abs(m * h - z) > 1e-9 * max(abs(z), h):
        raise ValueError(f"z = {z} is not on the step grid {h}")
    return m


def mpa_propagate(a: np.ndarray, dt: float, dmmap, L: float, M: int, n_iter: int,
                  z0: float, z1: float, block: int = 0, halo: int = 0, shift: int = 0) -> np.ndarray:
    """March long steps from z0 to z1 (both on the long-step grid)."""
    m0, m1 = _grid_index(z0, L), _grid_index(z1, L)
    for m in range(m0, m1):
        a = mpa_step(a, dt, dmmap, L, M, n_iter, m, block, halo, shift)
    return a


# --------------------------------------------------------------------------
# Split-step comparator, Eq. 4
# --------------------------------------------------------------------------

def ss_long_step(a0: np.ndarray, omega: np.ndarray, beta2: float, beta3: float,
                 sigma: float, gamma: float, L: float, M: int) -> np.ndarray:
    """Composite split-step over L with M steps, Eq. 4:
    A_SS(L) = e^{i L dz/2} Q^M e^{-i L dz/2} A(0), Q = e^{i N dz} e^{i L dz}.
    e^{i L h} is exact linear propagation over h (loss included, h may be
    negative); e^{i N h} A = A exp(i sigma |A|^2 h) solves the nonlinear part
    exactly."""
    dz = L / M
    a = linear_step(a0, omega, beta2, beta3, gamma, -dz / 2)
    for _ in range(M):
        a = linear_step(a, omega, beta2, beta3, gamma, dz)
        a = a * np.exp(1j * sigma * np.abs(a) ** 2 * dz)
    return linear_step(a, omega, beta2, beta3, gamma, dz / 2)


def ss_long_step_gain(a0: np.ndarray, omega: np.ndarray, beta2: float, beta3: float,
                      sigma: float, dmmap, zeta0: float, dz: float, steps: int) -> np.ndarray:
    """Split-step of Eq. 4 over `steps` steps of dz when G depends on z
    (distributed gain): every step is the symmetric product of Eq. 4,
    e^{i L dz/2} e^{i N dz} e^{i L dz/2}, and each linear half step propagates
    exactly over its own interval, multiplying by exp(int G) over it (zeta0 is
    the start's position in its amplifier period; the run stays inside it)."""
    a = a0
    for j in range(steps):
        z = zeta0 + j * dz
        for half, zs in ((0, z), (1, z + dz / 2)):
            g = float(gain_integral(dmmap, zs, dz / 2))
            a = paper_ifft(paper_fft(a) * np.exp(1j * beta_phase(omega, beta2, beta3, dz / 2) + g))
            if half == 0:
                a = a * np.exp(1j * sigma * np.abs(a) ** 2 * dz)
    return a


def ss_propagate(a: np.ndarray, dt: float, dmmap, dz: float, z0: float,
                 z1: float) -> np.ndarray:
    """Split-step from z0 to z1 with step dz: Eq. 4 applied to every run of
    steps that stays inside one span and ends at the next span boundary,
    amplifier or z1; lumped gain after a run ending on an amplifier.  With
    distributed gain the runs take ss_long_step_gain and the lumped gain is
    that of lumped_gain."""
    n = a.shape[0]
    omega = omega_grid(n, dt)
    j0, j1 = _grid_index(z0, dz), _grid_index(z1, dz)
    every = _amp_every(dmmap, dz)
    counts = [_steps_per(s, dz, "span") for s in dmmap.seg_len]
    period = sum(counts)
    j = j0
    while j < j1:
        s = span_of_long_step(dmmap, dz, j)
        # steps left in this span
        r = j % period
        acc = 0
        for c in counts[:s + 1]:
            acc += c
        run = min(acc - r, j1 - j)
        if every:
            run = min(run, every - (j % every))
        if _raman(dmmap)[0] > 0:
            if not every:
                raise ValueError("distributed gain needs amplifiers (z_amp > 0)")
            a = ss_long_step_gain(a, omega, dmmap.beta2[s], dmmap.beta3[s], dmmap.sigma[s], dmmap,
                                  (j % every) * dz, dz, run)
        else:
            a = ss_long_step(a, omega, dmmap.beta2[s], dmmap.beta3[s], dmmap.sigma[s],
                             dmmap.gamma, run * dz, run)
        j += run
        if every and j % every == 0:
            a = a * lumped_gain(dmmap)
    return a


def reference_propagate(a: np.ndarray, dt: float, dmmap, z0: float, z1: float,
                        steps0: int, rtol: float = 1e-12, max_doublings: int = 8):
    """Converged FP64 reference: split-step with Richardson extrapolation
    (4 A_{h/2} - A_h)/3, halving h until successive extrapolations agree to
    rtol (the paper's "numerically exact" solution was a very fine split-step
    run).  steps0 is the starting number of steps over [z0, z1].  Returns
    (A_ref, estimated relative error)."""
    span = z1 - z0
    steps = steps0
    prev_h = ss_propagate(a, dt, dmmap, span / steps, z0, z1)
    prev_x = None
    est = float("inf")
    for _ in range(max_doublings):
        steps *= 2
        cur_h = ss_propagate(a, dt, dmmap, span / steps, z0, z1)
        x = (4.0 * cur_h - prev_h) / 3.0
        if prev_x is not None:
            est = rel_l2(prev_x, x)
            if est < rtol:
                return x, est
        prev_x, prev_h = x, cur_h
    return prev_x, est
