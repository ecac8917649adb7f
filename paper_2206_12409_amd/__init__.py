"""MI355X-native hybrid volume-surface integral equation (VSIE) operator and solver.

The compute path is libvsie.so (HIP kernels for gfx950 behind the C ABI of include/vsie.h);
this package only builds it and binds it (vsie.Operator).
"""
from .vsie import Net, Operator, ProductGraph, VsieError, default_options, dense_lu_solve, load  # noqa: F401
