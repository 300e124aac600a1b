"""FP64 CPU oracle for the paper's discrete acoustic operator H_a and its adjoint.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package.  The GPU library never imports, links or
calls it, and this package imports nothing from the library.

Paper: Javaherian & Holman, "Direct quantitative photoacoustic tomography for
realistic acoustic media" (arXiv 1810.11685).

* `kspace.forward`   - Section 3.2.3 ("Numerical computation of the acoustic
  forward operator"): the k-space PSTD loop (eqs num-vel, num-rho, num-p,
  num-m) with the additive source of eq s1, discretised operators of
  Section 3.2.2 (eq grr, Y_abs, Y_dis, eq dis-pml).
* `kspace.adjoint`   - exact transpose of `forward` (reverse mode, step by step).
* `kspace.adjoint_paper` - the paper's own adjoint recursion, eq t41 with the
  pairwise-summed adjoint source of eq adj_data (Section 3.2.4, Lemma 2).
* `dense`            - brute force on tiny grids: explicit DFT matrices, the
  block one-step matrix T of eq Tprod (with D, E, G of eqs D4, E, G4) and the
  dense H_a of Definition 4, for cross-checking the three routines above.
"""
from .kspace import (Operators, forward, adjoint, adjoint_paper, gradient, sensor_taps,
                     alpha0_np, tau_eta, stability_limit)

__all__ = ["Operators", "forward", "adjoint", "adjoint_paper", "gradient", "sensor_taps",
           "alpha0_np", "tau_eta", "stability_limit"]
