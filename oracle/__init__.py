"""CPU oracle for the FMM-LU hot path (test infrastructure, not product code).

A plain, slow, obviously correct float64 implementation of what the GPU library
computes, written from the paper (Sushnikova, Greengard, O'Neil, Rachh, "FMM-LU:
A fast direct solver for multiscale boundary integral equations in three
dimensions"). It exists only to check the GPU path: nothing in the product
package imports, links or calls it. Only the test-suite, the smoke entry point
and the CPU-baseline leg of the benchmark may use it.

Modules
  kernel   Helmholtz Green's function and combined-field kernel entries (Section 3).
  dense    dense system matrix, dense LU solve, exact matvec (Section 3, eq. disc3).
  tree     level-restricted adaptive octree (Section 4, opening; Section 4.4).
  idqr     greedy column-pivoted QR interpolative decomposition (Section 4.1, Definition 1).
  rss      recursive strong skeletonization with dense bookkeeping, forward and
           adjoint solve of the factored inverse (Sections 4.1-4.4, 5.1-5.2).
  farfield far-field pattern and gradients of a far-field loss (Section 6.3).

Every function cites the passage it follows by section or equation label. Where
the paper is silent, the reading taken is stated in the docstring.
"""
