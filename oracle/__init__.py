"""Plain FP64 CPU oracle for the angular-multigrid DG transport solver of
Lathouwers & Perko, "An Angular Multigrid Preconditioner for the Radiation
Transport Equation with Forward-Peaked Scatter" (arXiv 2010.04559).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The HIP library under ``paper_2010_04559_amd`` never imports,
links or calls anything here, and nothing here imports that package: the two
share no kernels, tables, helpers or constant generators.

Everything is written for clarity, in the paper's notation and order, in
float64 numpy.  There is no blocking, fusion or reordering beyond what the
definitions need; library primitives (dense solves, matrix products) serve as
single steps.

Modules
-------
angular    hierarchical spherical-triangle patches, Lin and Const bases, quadrature,
           angular matrices, Legendre scatter kernel, prolongation
           (Sections 2.1-2.2, 4.1, 5.2, 5.5)
spatial    trilinear/bilinear nodal DG matrices on a Cartesian mesh
           (Section 2.3)
transport  the weak form (eq. complete), the upwind flux, the transport
           sweep, the scatter source, right-hand sides and detector weights
           (Sections 2.3, 3, 5.2)
multigrid  direct-discretisation level operators, the coarsest-level block
           Gauss-Seidel sweep and the V-cycle of Fig. lmg (Sections 4, 5.2)
krylov     restarted, right-preconditioned GMRES(m)
adjoint    transposed operators, the adjoint solve and the detector-response
           gradient with respect to per-cell sigma_t and sigma_s

Parity status: every function is pinned by the ``-m "not gpu"`` tests
(closed forms, invariants, brute-force dense solves, the paper's mesh
counts) except the Krylov iteration counts themselves, which the paper does
not fix for this configuration (its counts are BiCGStab with Fokker-Planck
moments): "parity unpinned" for iteration counts, checked only as trends.
"""
