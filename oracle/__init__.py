"""Plain, slow CPU FP64 oracle of the MGCG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import or call this package; only the test-suite,
the bench's CPU-baseline leg and the smoke check use it.  It shares no code,
tables or constants with the HIP library: every element matrix, operator and
gradient here is computed afresh from the paper's formulas.

What it computes (the plain definitions, in FP64):

* ``fem``      element stiffness of Lagrange (degree 1-3) and serendipity
               (degree 2-3) hexahedra by Gauss quadrature (Sec. 2.1),
               including the sub-element matrices of the multiresolution
               element (Sec. 3.3, unnumbered split of the integral, and
               eq. (7));
* ``assemble`` SIMP moduli (eq. (1) / (7)) and the sparse global K with the
               supported DOFs removed (Sec. 2, Sec. 6.1);
* ``solve``    u = K_ff^{-1} f_f by a dense or sparse direct factorisation,
               compliance f^T u (problem (2)) and the density gradient
               (Sec. 3.4, without the design-variable chain factor);
* ``multigrid`` explicit sparse prolongation P (trilinear interpolation,
               Sec. 2.3) and the Galerkin coarse operators P^T A P, the
               weighted-Jacobi sweep and Algorithm 1 applied recursively
               (the preconditioner M as a plain linear operator), plus the
               paper's preconditioned CG used as a reference solver where a
               direct factorisation is too large;
* ``projection`` the weighted-average projection of design variables onto
               densities (Sec. 3.2 eq. (5), weights of Sec. 2.2 eq. (4); the
               density filter when both lattices coincide) and its transpose,
               the chain rule of Sec. 3.4;
* ``slp``      the SLP step of Sec. 4: the LP subproblem with the volume
               constraint and the trust region (a fractional knapsack), the
               artificial problem, and the step control of Algorithm 2;
* ``threshold`` the density thresholding of Sec. 5: rounding, the
               density-value strategy, the angle condition, the strategy
               based on the gradient of the Lagrangian and the Heaviside
               projection with its volume-preserving threshold;
* ``fixing``   the choice of fixed variables of Sec. 6.1: void and solid
               elements, the surrounded rule, fixed design variables and
               suppressed nodes of the raised degree.

Parity status of every function is listed in its module docstring.
"""
