"""MI355X-native fourth-order cut-cell multigrid Poisson solver.

`inputs` holds the seeded workload generators; `_lib` is the ctypes binding of
the HIP library (built in-tree by `build`).  Importing the package loads
nothing: the library is loaded on first use of `_lib`.
"""
__all__ = ["inputs"]
