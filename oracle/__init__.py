"""CPU FP64 oracle for the directional FMM matvec (test infrastructure only).

This package is the checker, not the product.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it; the library
under ``paper_1311_4257_amd`` never does, and the two share no code.

Modules:
  kernel     the Helmholtz Green's function and the plain O(N^2) sum (Eq. 1)
  tree       octree, near fields, interaction lists, wedges (Section 2.2)
  operators  directional skeletons (a, b, D) of Eq. 2 by pivoted QR
  fmm        the evaluation pass of Algorithm 1 plus the near-field sum

Everything is float64 / complex128 NumPy.  Readings of places where the
paper is silent or garbled are stated in each function's docstring.
"""
