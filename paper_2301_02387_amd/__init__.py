"""MI355X hot path of MCTDHF on an adaptive finite-element mesh.

Thin Python binding over the C ABI of ``libmh.so`` (declared in
``include/mh.h``): argument marshalling only.  Device arrays are torch
tensors on the GPU (complex128 orbital arrays, float64 Poisson columns);
every computation runs in the library's HIP kernels.  There is no CPU
fallback: importing works without a GPU, but every call needs the built
library and a GPU.
"""
from ._lib import (Mesh, Operator, MHError, lib_path, load_library, set_allocator,  # noqa: F401
                   MH_OK, MH_NOT_CONVERGED)

__all__ = ["Mesh", "Operator", "MHError", "lib_path", "load_library", "set_allocator"]
