"""Plain, slow, FP64 CPU oracle of the one-way Helmholtz propagator step.

This package is TEST INFRASTRUCTURE.  It exists to check the GPU library
against the paper (Keefe, McDaniel, Cubillos, Zilberter, Madden, "A vector
Helmholtz electromagnetic wave propagator for inhomogeneous media").  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the GPU library and imports nothing from it.

Modules
-------
stencil   13-point 4th-order finite-difference stencils (Sec. 4.1)
fit       AAA / AAA-Lawson rational fit of exp(iK sqrt(1+z)) and its partial
          fractions (Sec. 2 eqs. rational approximation / pf_expan_eq, Sec. 3.1)
operator  coefficient fields and the operator matrix Zbar (Sec. 2 eq. Z_bar_eq)
precond   free-space preconditioner as a Sylvester solve diagonalised by DST-I
          (Sec. 4.2.1-4.2.2, eqs. Z_bar_fs_def, fs_sylvester)
gmres     right-preconditioned GMRES with Householder Arnoldi (Sec. 4.2)
step      one propagation step and a propagation loop (Sec. 2 eqs. Wk_define,
          approx_prop, W_k_def)
sqrt_form pseudo-differential form: Cauchy-integral partial fractions of
          sqrt(1+z) (Sec. 3.2, Appendix A) and an RK4 integrator in z
physics   closed forms used as pins (Sec. 3 eq. exp_prop_planewave,
          Sec. 5.2 eq. eq_ft_gaussian)
"""
