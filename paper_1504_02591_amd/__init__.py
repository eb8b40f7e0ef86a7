"""MI355X (gfx950) iterative Fourier-space reconstruction with wide-angle RSD.

The compute path is the HIP library built from csrc/ (C ABI in include/recon.h);
`native` is its ctypes binding.  Importing the package does not load the library.
"""
__all__ = ["native", "build"]
