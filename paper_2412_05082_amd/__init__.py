"""MI355X-native C0IP biharmonic operator, vertex-patch smoother, multigrid
and flexible GMRES (arXiv 2412.05082), behind the C ABI of libc0ip.so.

The Python layer only marshals arguments: every step of the operator,
smoother, V-cycle and Krylov solve runs in the library's HIP kernels.
"""
from .binding import (C0IP_F32, C0IP_F64, Batch, C0ipError, KrylovOpts, MeshDesc, MgOpts, Problem, SolveInfo,
                      host_matrices_1d, host_patch_inverse, host_patch_inverse_exact, lib_path, load_library)

__all__ = ["C0IP_F32", "C0IP_F64", "Batch", "C0ipError", "KrylovOpts", "MeshDesc", "MgOpts", "Problem", "SolveInfo",
           "host_matrices_1d", "host_patch_inverse", "host_patch_inverse_exact", "lib_path", "load_library"]
