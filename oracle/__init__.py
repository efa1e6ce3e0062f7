"""FP64 CPU oracle for the stabilised natural-convection state solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product (the HIP library in
``paper_1508_04596_amd``) never imports, links or runs anything from here, and
this package imports nothing from the product; the two share only the seeded
input generators, which hold none of the method's arithmetic.

Contents:

* ``fe_oracle.c`` -- the element loops in plain C: residual, J v, J^T w (via the
  element Jacobian transposed), lambda^T dR/dgamma, element Jacobians.
* ``core`` -- ctypes wrappers and the build step for that library.
* ``solve`` -- sparse assembly of the Jacobian from element Jacobians, the damped
  Newton iteration with the quadratic L2 line search (exact linear solves), the
  adjoint solve and the thermal-compliance objective.
"""
from .core import (build_oracle, residual, jvp, jtvp, dR_dgamma, element_jacobians,  # noqa: F401
                   element_residual, element_dR_dgamma, material, taus, gauss_points,
                   num_threads, set_num_threads, set_frozen_tau)
