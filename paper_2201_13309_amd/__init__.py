"""MI355X (gfx950) wire-scan depth reconstruction.

The work happens in libdr.so (HIP kernels + C++ runtime, C ABI in
include/dr.h); ``paper_2201_13309_amd.dr`` is its ctypes binding.  This
package import does not load the library, so that the build step can run
first; importing ``paper_2201_13309_amd.dr`` loads it or fails loudly.
"""
__all__ = ["dr", "build"]
