"""CPU oracle for the fourth-order cut-cell multigrid Poisson solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64
numpy/scipy restatement of what the method computes, written from the
paper (Qian, Li, Tan, Zhang, "A fourth-order, multigrid cut-cell method
for solving Poisson's equation in three-dimensional irregular domains",
arXiv 2410.05865).  It shares no code with the HIP library and must only
be imported by the tests, by the smoke check and by the CPU-baseline leg
of the benchmark.  The product path never calls it.

Modules
  fields      analytic fields and their exact cell / face averages
  quadrature  high-order quadrature on implicitly defined cut cells
  geometry    cell classification, moments, face apertures (Sec. 2.2)
  merging     small-cell merging (Sec. 4.2, MAP-3 and the BFS fallback)
  discretize  regular rows with ghost cells (Sec. 2.3), FV-PLG rows
              (Secs. 2.3, 4.1), assembly of L and r = f - N g (Sec. 2.4)
  multigrid   SMO-1, SMO-2 (LU-correction), transfers, VCycle and the
              Multigrid driver (Sec. 5.3)

Functions whose result is not pinned by a closed form, an invariant or
an independent computation say "parity unpinned" in their docstring.
"""
