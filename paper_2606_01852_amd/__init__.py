"""MI355X (gfx950) tensor-network path executor.

The product is the C-ABI library ``libtnc.so`` (HIP kernels + C++ planner
and executor, declared in include/tnc.h); ``paper_2606_01852_amd.tnc`` is its
ctypes binding.  Importing this package loads nothing; the binding loads the
library on first use and fails loudly if it has not been built.
"""
__all__ = ["tnc", "build"]
