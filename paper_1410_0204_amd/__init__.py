"""MI355X-native transport-matrix time stepping (Metos3D method, arXiv 1410.0204).

The compute path is the HIP library ``libtmm.so`` (C ABI in include/tmm.h);
``paper_1410_0204_amd.tmm`` is its ctypes binding.  Submodules are imported
on demand so that importing the package does not touch the GPU.
"""

__all__ = ["tmm", "autograd", "drivers"]
