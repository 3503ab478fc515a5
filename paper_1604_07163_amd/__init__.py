"""MI355X (gfx950) geometric-multigrid-preconditioned CG for -div(k grad phi) = f.

The compute path is libgmg.so (HIP kernels behind the C ABI in include/gmg.h);
`gmg.Solver` is its ctypes binding and `autograd.DiffusionSolve` the
differentiable wrapper.  Importing this package does not load the library;
the first solver call does, and raises if it is not built.
"""
__all__ = ["gmg", "autograd", "inputs"]
