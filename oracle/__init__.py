"""Plain FP64 CPU oracle for the two-level DD-alpha-AMG hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never calls it, and the two share no code:
the only common inputs come from the seeded generators in `workloads/`.

Everything here is written from the paper's description of the method
(Ishikawa & Kanamori, "Porting DDalphaAMG solver to K computer", Sec. 2:
Eq. (1) aggregation with chirality split, Eq. (2) Galerkin coarse operator,
Eqs. (3)-(4) restriction and prolongation, Eq. (5) the preconditioner; the
SAP smoother with even-odd minimal-residual block solves; the even-odd coarse
GMRES; the flexible GMRES outer solver; the adaptive setup) and the standard
Wilson-clover operator of the DD-alpha-AMG method the paper ports.  Arrays
are complex128 and the arithmetic is numpy FP64 throughout.

Modules
  lattice : geometry, aggregate / block / parity maps, shifts with the t boundary sign
  gamma   : the chiral-basis gamma matrices
  dirac   : clover term, packed Hermitian storage, inverse clover, D and its block pieces
  amg     : Gram-Schmidt, P, R, coarse operator, coarse GMRES, SAP, V-cycle, FGMRES, setup
"""
