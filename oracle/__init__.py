"""Plain serial FP64 CPU oracle for Krylov-subspace-enhanced Parareal applied to
the linear 2D acoustic-advection system (Ruprecht & Krause, "Explicit
parallel-in-time integration of a linear acoustic-advection system").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or pre/post-processing).

Layout of a state: ``numpy.ndarray`` of shape ``(3, nz, nx)``, float64, field
order (u, w, p) -- the paper's (u, v, pi) on the x-y plane, renamed to the
x-z plane -- with x fastest.  Periodic in both directions; cell-centred
points x_i = (i + 1/2) dx, z_j = (j + 1/2) dz on [0, 1]^2.

Modules
  operators   flux-form spatial operators (Section 3, flux-difference formula)
  propagators fine RK-3 propagator F and split-explicit coarse propagator G
              (Section 3.2)
  kse         subspace update (pivoted Householder QR, Section 2.2), the
              modified coarse propagator K (eq. modifiedCoarse / eq. Genhance),
              Algorithm 2 (KSE-Parareal), Algorithm 1 (original Parareal) and
              the relative l2 error (eq. errorDef)

Every function is pinned by ``tests/test_oracle_*.py`` against facts that do
not come from this code: Fourier symbols of the stencils (closed-form
amplification factors), convergence orders against calculus, LAPACK's
pivoted QR invariants, the exactness of Parareal after k iterations, and a
dense brute-force run on an 8x8 grid.
"""

from .operators import Params, rhs_fine, coarse_slow_tendency, acoustic_substep
from .propagators import fine_F, coarse_G, serial_fine
from .kse import (subspace_update, kse_apply, kse_parareal, parareal,
                  rel_l2)

__all__ = [
    "Params", "rhs_fine", "coarse_slow_tendency", "acoustic_substep",
    "fine_F", "coarse_G", "serial_fine", "subspace_update", "kse_apply",
    "kse_parareal", "parareal", "rel_l2",
]
