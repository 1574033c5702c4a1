"""FP64 CPU oracle of the massively parallel algorithm (MPA) and of split-step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything in this package: only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library.

Every function follows one passage of Korotkevich & Lushnikov,
"Proof-of-concept implementation of the massively parallel algorithm for
simulation of dispersion-managed WDM optical fiber systems"
(arXiv:1101.0086), cited by equation number (Eq. 1 ... Eq. 7, in order of
appearance) or by the numbered MPA steps 1-7.

Parity status of each function (what pins it, see tests/test_oracle_*.py):

* ``paper_fft`` / ``paper_ifft``: brute-force DFT with the e^{+i omega t}
  kernel of the Fourier transform definition.
* ``linear_step``: Gaussian closed form (beta3 = 0) and the exact centroid
  drift from the moment equation of Eq. 1 (beta3 != 0).
* ``mpa_long_step``: sigma = 0 exactness; the beta = 0 closed forms
  (first iterate = Euler over L, exact rational second iterate, Cayley
  limit); n -> infinity equals the sequential implicit trapezoid; SPM with
  loss; soliton; the analytic MPA/SS error ratio 2 of Eqs. 5 and 7.
* ``mpa_blocked_long_step``: block = N reproduces the full window bitwise;
  shift equivariance; sigma = 0 blocked error below the halo bound; with
  windows shifted against their cores, a one-sided group delay that the
  centred windows cannot hold is held by the shifted ones.
* ``parallel.mpa_long_step_parallel`` (the paper's decomposition of a long
  step over z-nodes and harmonic ranges, for the CPU baseline): equals
  ``mpa_long_step`` to rounding.
* ``ss_long_step`` / ``ss_propagate``: linear closed forms; exact SPM
  kick; second order; unitarity; time reversibility.
* ``ss_long_step_gain`` (split-step with distributed gain): the exact linear
  solution at sigma = 0, the energy balance exp(2 int G) to rounding, and
  the uniform-loss split-step when the distributed gain is zero.
* ``mpa_propagate``: marching and resume identity; lumped gain restores the
  span loss exactly.
* ``mpa_long_step_vjp`` / ``mpa_long_step_vjp_nodes`` /
  ``mpa_blocked_long_step_vjp`` / ``mpa_propagate_vjp`` (module
  ``adjoint``): gradients of a real loss with respect to the input field,
  sigma, beta2 and beta3 (per span), pinned by central finite differences
  of the forward functions above, across a span change, an amplifier, the
  dispersion-dependent roll-off and long steps that cross span boundaries
  (``step_weights``: also pinned against ``step_coefficients``).
* the FP32 rounding pattern of the GPU path has no oracle: FP32 results
  are compared with this FP64 oracle ("parity unpinned" for the FP32
  rounding pattern itself).
"""
from .nlse import (DMMapSpec, paper_fft, paper_ifft, omega_grid, beta_phase,
                   linear_step, mpa_long_step, mpa_blocked_long_step,
                   block_partition, block_taper, block_mask, halo_rate, group_delay_range,
                   halo_excursion, mpa_step, mpa_propagate, ss_long_step,
                   ss_long_step_gain,
                   ss_propagate, reference_propagate, if_trapezoid_long_step,
                   span_of_long_step, rel_l2)
from .adjoint import (mpa_long_step_vjp, mpa_long_step_vjp_nodes, mpa_blocked_long_step_vjp,
                      mpa_propagate_vjp, block_mask_grad, step_weights)

__all__ = ["DMMapSpec", "paper_fft", "paper_ifft", "omega_grid", "beta_phase",
           "linear_step", "mpa_long_step", "mpa_blocked_long_step",
           "block_partition", "block_taper", "block_mask", "halo_rate", "group_delay_range",
           "halo_excursion", "mpa_step", "mpa_propagate", "ss_long_step",
           "ss_long_step_gain",
           "ss_propagate", "reference_propagate", "if_trapezoid_long_step",
           "span_of_long_step", "rel_l2", "mpa_long_step_vjp", "mpa_blocked_long_step_vjp",
           "mpa_long_step_vjp_nodes", "mpa_propagate_vjp", "block_mask_grad", "step_weights"]
