"""CPU FP64 oracle of the symmetry-preserving JFNK hot path.

ORACLE - TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it.  The HIP library never calls,
links or imports anything here, and this package imports nothing from the HIP
library: the two share no code.  Inputs reach both from the seeded generators in
``paper_2007_10411_amd.inputs``, which hold none of the method's arithmetic.

Modules:
  stencil  - Deslauriers-Dubuc derivative stencil from the refinement relation (section 2.3)
  model    - F(u), R(u), f(u^n), Jv (equations 1-5 and 9, sections 2.2-2.5)
  precond  - physics-based field-block preconditioner (section 2.5.2)
  krylov   - flexible restarted GMRES and inexact Newton (section 2.5.1, equation 8)
  net      - the learned convolutional preconditioner, forward and backward, FP64
"""
