"""FP64 CPU oracle for mixed-precision DIRK time stepping of 3-D finite-difference PDEs.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers or constant tables); both sides take
their inputs from the ``workloads`` module.

What it computes (all float64, numpy/scipy):
  * operators.py   -- the semi-discrete operator K of du/dt = K u (Section
                      "Problem setting and solver design"): 7-point heat Laplacian
                      and first-order-upwind advection-diffusion, CSR.
  * tableaus.py    -- Butcher tableaus split as A = A^(h) + A^(eps)
                      (Section "Method stability in the context of mixed precision"),
                      the mixed midpoint rule with corrections (Figure fig_Aq_rat,
                      Appendix A), 4s3pA/B/C (Tables ButchertabA/B/C), and the
                      configuration SDIRKs; the stability function R(z).
  * dirk.py        -- the DIRK step of eq. (RKstep) with exact stage solves
                      (dense LU, sparse LU or the oracle's own FP64 Krylov).
  * krylov.py      -- plain FP64 CG, right-preconditioned GMRES(m) and block
                      Jacobi (used for large grids and for solver pins).
  * nonlinear.py   -- the same DIRK for du/dt = K u + g + R(u) with a pointwise
                      cubic reaction R, Newton stage solves (exact Jacobian).
  * closed_form.py -- modal closed forms: sine modes / DST-I for the Dirichlet
                      Laplacian, DFT for the periodic operator; u_N = R(tau lam)^N.
Every function cites the passage it follows.  Parity status of each part is
stated in its module docstring; the mixed-precision GPU paths have no oracle of
their own beyond the FP64 result and the stated tolerances.
"""
from . import operators, tableaus, dirk, krylov, closed_form, nonlinear  # noqa: F401
